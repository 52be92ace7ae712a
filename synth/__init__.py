"""Seeded synthetic inputs for the FDAS hot path.

This module only *draws* inputs: white Gaussian time series with injected
binary-pulsar signals, their real FFT and the median-power normalisation that
turns them into the complex spectrum the correlation consumes.  It holds none
of the correlation arithmetic (no templates, no response function, no plane,
no peaks), so the CPU oracle and the GPU path can both take their inputs from
here without sharing any of the method.

Stand-in for the paper's data: the paper draws ~20,000 filterbank files with
SIGPROC ``fake`` (Section "Generating synthetic data", Table 2) and one GMRT
observation (Section "Real data"); neither is available, so every spectrum
here is synthetic, drawn from ``numpy.random.Generator(PCG64(SeedSequence(
[12205, config, trial])))``.

Conventions
-----------
* Time series x[n], n in [0, N_t), sample time ``tsamp``; T = N_t * tsamp.
* A real signal a*cos(2 pi (f t + fdot t^2 / 2) + phi) has initial Fourier
  frequency r0 = f T and drift z = fdot T^2 (Eq. 1 defines z as the drift in
  Fourier bins); its mean Fourier frequency is r_bar = r0 + z / 2.
* Spectrum: X = rfft(x), keep k in [0, N_t/2) (Nyquist dropped), X[0] = 0
  (the DC bin carries the series mean, Section "IEEE-754 Half vs bfloat16"),
  then divide by sqrt(median_{k>=1} |X[k]|^2 / ln 2) so that noise powers are
  Exp(1) (the paper observes chi^2_2-shaped noise, Section "Noise properties").
  Noise-free inputs use the declared sigma instead (divide by sqrt(N_t)).
* Output dtype is complex64: the real FFT stays in single precision in the
  paper (Section "Updating the pipeline to bfloat16"), and this single-precision
  array is the common input of every path.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PAPER_SEED = 12205

# Workload shapes.  z grids are z_j = z_min + j * z_step.
CONFIGS = {
    1: dict(name="tiny", n_t=2 ** 17, tsamp=64e-6, z_min=-16.0, z_step=2.0,
            n_z=17, n_taps=64, seg_len=1024, threshold=20.0),
    2: dict(name="single-DM", n_t=2 ** 23, tsamp=64e-6, z_min=-100.0,
            z_step=2.0, n_z=101, n_taps=256, seg_len=8192, threshold=45.0),
    3: dict(name="batched", n_spec=256, n_t_min=2 ** 20, n_t_max=2 ** 23,
            tsamps=(64e-6, 128e-6, 256e-6, 512e-6), frac_pulsar=0.1, z_min=-100.0,
            z_step=2.0, n_z=101, n_taps=256, threshold=45.0),
    5: dict(name="wide", n_t=2 ** 24, tsamp=64e-6, z_min=-200.0, z_step=2.0,
            n_z=201, n_taps=512, seg_len=16384, threshold=45.0),
}

DUTY = 0.05            # Gaussian pulse FWHM as a fraction of the period
N_HARM = 8             # harmonics injected per pulsar
NYQ_GUARD = 0.95       # drop harmonics whose frequency reaches 0.95 f_Nyq


def rng(config: int, trial: int) -> np.random.Generator:
    """The one seeded generator every synthetic input is drawn from."""
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([PAPER_SEED, int(config), int(trial)])))


@dataclass
class Pulsar:
    """An injected binary pulsar (fundamental f, drift fdot, harmonics)."""
    f: float                     # Hz at t = 0
    fdot: float                  # Hz / s
    amps: list                   # a_h for h = 1..len(amps)
    phases: list                 # phi_h
    p1: float                    # declared noise-free matched power of h = 1

    def z(self, T: float, h: int = 1) -> float:
        return h * self.fdot * T * T

    def r_bar(self, T: float, h: int = 1) -> float:
        """Mean Fourier frequency of harmonic h (bins)."""
        return h * (self.f * T + 0.5 * self.fdot * T * T)


@dataclass
class Spectrum:
    spec: np.ndarray             # complex64, N = n_t / 2 bins
    n_t: int
    tsamp: float
    pulsars: list = field(default_factory=list)

    @property
    def T(self) -> float:
        return self.n_t * self.tsamp


def pulse_harmonic_weights(n_harm: int = N_HARM, duty: float = DUTY):
    """Fourier amplitudes c_h of a Gaussian pulse with FWHM = duty * period."""
    return [math.exp(-(math.pi * h * duty) ** 2 / (4.0 * math.log(2.0)))
            for h in range(1, n_harm + 1)]


def add_signal(x: np.ndarray, tsamp: float, p: Pulsar) -> None:
    """x += sum_h a_h cos(2 pi h (f t + fdot t^2 / 2) + phi_h), in place (FP64)."""
    t = np.arange(x.size, dtype=np.float64) * tsamp
    cyc = p.f * t + 0.5 * p.fdot * t * t          # cycles of the fundamental
    for h, (a, ph) in enumerate(zip(p.amps, p.phases), start=1):
        if a == 0.0:
            continue
        c = h * cyc
        c -= np.floor(c)                             # keep the phase argument small
        x += a * np.cos(2.0 * np.pi * c + ph)


def to_spectrum(x: np.ndarray, sigma: float | None = None) -> np.ndarray:
    """Real FFT, drop Nyquist, zero DC, normalise; returns complex64.

    sigma=None: median-power normalisation (noise powers become Exp(1)).
    sigma=s:    divide by s * sqrt(N_t) (noise-free inputs of declared sigma).
    """
    n_t = x.size
    X = np.fft.rfft(x)[: n_t // 2]
    X[0] = 0.0
    if sigma is None:
        med = np.median(X[1:].real ** 2 + X[1:].imag ** 2)
        X /= math.sqrt(med / math.log(2.0))
    else:
        X /= sigma * math.sqrt(n_t)
    return X.astype(np.complex64)


def draw_pulsar(g: np.random.Generator, T: float, tsamp: float,
                p_range=(1e-3, 10e-3), z_range=(-80.0, 80.0),
                p1_range=(10.0, 4000.0), n_t: int = 0) -> Pulsar:
    """A binary pulsar as in the single-DM workload: P ~ U, z ~ U, 8 harmonics,
    5 % duty cycle, fundamental matched power P1 ~ log-U[10, 4000]."""
    period = g.uniform(*p_range)
    z1 = g.uniform(*z_range)
    p1 = math.exp(g.uniform(math.log(p1_range[0]), math.log(p1_range[1])))
    phases = list(g.uniform(0.0, 2.0 * math.pi, size=N_HARM))
    f = 1.0 / period
    fdot = z1 / (T * T)
    c = pulse_harmonic_weights()
    a1 = math.sqrt(4.0 * p1 / n_t)
    f_nyq = 0.5 / tsamp
    amps = []
    for h in range(1, N_HARM + 1):
        fmax = h * max(f, f + fdot * T)
        amps.append(0.0 if fmax >= NYQ_GUARD * f_nyq else a1 * c[h - 1] / c[0])
    return Pulsar(f=f, fdot=fdot, amps=amps, phases=phases, p1=p1)


def config1_series(trial: int = 0):
    """The tiny workload's time series (float64) and its pulsar: 2^17 samples
    at 64 us, one sinusoid f = 137.3 Hz, z = +6.4.

    Amplitude reading: noise-free matched power 200 (matched-filter amplitude
    SNR sqrt(2 * 200) = 20), i.e. a = sqrt(4 * 200 / N_t) for unit-sigma noise.
    """
    c = CONFIGS[1]
    n_t, tsamp = c["n_t"], c["tsamp"]
    T = n_t * tsamp
    g = rng(1, trial)
    x = g.standard_normal(n_t)
    p = Pulsar(f=137.3, fdot=6.4 / (T * T), amps=[math.sqrt(4.0 * 200.0 / n_t)],
               phases=[float(g.uniform(0.0, 2.0 * math.pi))], p1=200.0)
    add_signal(x, tsamp, p)
    return x, p


def config1(trial: int = 0) -> Spectrum:
    """Tiny workload spectrum (config1_series through to_spectrum)."""
    c = CONFIGS[1]
    x, p = config1_series(trial)
    return Spectrum(to_spectrum(x), c["n_t"], c["tsamp"], [p])


def config2_series(trial: int = 0, noise: bool = True):
    """The single-DM workload's time series (float64) and its pulsar: 2^23
    samples at 64 us, one 8-harmonic binary pulsar."""
    c = CONFIGS[2]
    n_t, tsamp = c["n_t"], c["tsamp"]
    T = n_t * tsamp
    g = rng(2, trial)
    x = g.standard_normal(n_t) if noise else np.zeros(n_t)
    p = draw_pulsar(g, T, tsamp, n_t=n_t)
    add_signal(x, tsamp, p)
    return x, p


def config2(trial: int = 0, noise: bool = True) -> Spectrum:
    """Single-DM workload spectrum (config2_series through to_spectrum)."""
    c = CONFIGS[2]
    x, p = config2_series(trial, noise)
    return Spectrum(to_spectrum(x, None if noise else 1.0), c["n_t"], c["tsamp"], [p])


def config5(trial: int = 0) -> Spectrum:
    """Wide workload: 2^24 samples at 64 us, 16 pulsars (P 1-20 ms, |z| <= 180)."""
    c = CONFIGS[5]
    n_t, tsamp = c["n_t"], c["tsamp"]
    T = n_t * tsamp
    g = rng(5, trial)
    x = g.standard_normal(n_t)
    ps = [draw_pulsar(g, T, tsamp, p_range=(1e-3, 20e-3), z_range=(-180.0, 180.0),
                      n_t=n_t) for _ in range(16)]
    for p in ps:
        add_signal(x, tsamp, p)
    return Spectrum(to_spectrum(x), n_t, tsamp, ps)


def noise_spectrum(n_bins: int, config: int = 0, trial: int = 0) -> np.ndarray:
    """Noise-only normalised spectrum of n_bins bins (series of 2 * n_bins)."""
    g = rng(config, trial)
    return to_spectrum(g.standard_normal(2 * n_bins))


def random_spectrum(n_bins: int, seed: int) -> np.ndarray:
    """Complex Gaussian bins (unit mean power), complex64; for shape/edge tests."""
    g = rng(900, seed)
    s = (g.standard_normal(n_bins) + 1j * g.standard_normal(n_bins)) / math.sqrt(2.0)
    return s.astype(np.complex64)


def complex_chirp_spectrum(n_t: int, r0: float, z: float, amp: float = 1.0, w: float = 0.0):
    """Noise-free spectrum of amp * exp(2 pi i (r0 u + z u^2 / 2 + w u^3 / 6)), u = n / n_t.

    Full complex FFT (a complex chirp has no mirror image), divided by sqrt(n_t)
    (declared sigma 1), first n_t / 2 bins kept, complex64.
    """
    u = np.arange(n_t, dtype=np.float64) / n_t
    cyc = r0 * u + 0.5 * z * u * u + w * u * u * u / 6.0
    cyc -= np.floor(cyc)
    x = amp * np.exp(2j * np.pi * cyc)
    X = np.fft.fft(x)[: n_t // 2] / math.sqrt(n_t)
    return X.astype(np.complex64)


def refine_offsets(n: int, trial: int = 0):
    """Seeded candidate offsets for refinement: dr ~ U[-0.5, 0.5], dz ~ U[-1, 1]."""
    g = rng(4, trial)
    return g.uniform(-0.5, 0.5, size=n), g.uniform(-1.0, 1.0, size=n)


@dataclass
class Trial:
    """One spectrum of the batched workload: its place in the packed tensor."""
    offset: int                  # first bin in the packed spectra
    n_bins: int
    n_t: int
    tsamp: float
    pulsar: Pulsar | None

    @property
    def T(self) -> float:
        return self.n_t * self.tsamp


def chirp_z_dft_head(x, n_out: int):
    """Bins 0 .. n_out - 1 of the length-N DFT X[k] = sum_n x[n] exp(-2 pi i n k / N)
    of a real or complex torch tensor x (any N, any device), complex128.

    Bluestein's chirp-z form: with n k = (n^2 + k^2 - (k - n)^2) / 2 and the
    chirp c[m] = exp(-i pi m^2 / N), X[k] = c[k] sum_n (x[n] c[n]) conj(c[k - n]),
    a linear convolution that a cyclic one of power-of-two length M >= 2N - 1
    computes without wrap-around, so only power-of-two FFTs run whatever N is.
    c[m] depends on m^2 mod 2N only, which is reduced exactly in integers
    before the angle is formed.
    """
    import torch
    N = int(x.numel())
    dev = x.device
    M = 1 << (2 * N - 2).bit_length()
    m = torch.arange(N, dtype=torch.int64, device=dev)
    ang = (m * m % (2 * N)).to(torch.float64) * (-math.pi / N)
    c = torch.polar(torch.ones_like(ang), ang)
    del m, ang
    a = torch.zeros(M, dtype=torch.complex128, device=dev)
    a[:N] = x.to(torch.complex128) * c
    b = torch.zeros(M, dtype=torch.complex128, device=dev)
    b[:N] = c.conj()
    if N > 1:
        b[M - N + 1:] = c[1:].conj().flip(0)
    fa = torch.fft.fft(a)
    del a
    fa *= torch.fft.fft(b)
    del b
    y = torch.fft.ifft(fa)[:n_out]
    return c[:n_out] * y


def _device_spectrum(n_t: int, tsamp: float, pulsars, seed: int, device, any_length: bool = False):
    """Gaussian series plus pulsars on the device (torch, FP64), then the
    to_spectrum recipe: real FFT, Nyquist dropped, DC zeroed, median
    normalisation; complex64.  any_length: the transform by chirp_z_dft_head
    (power-of-two FFTs only), so that no FFT plan is built for the length
    itself."""
    import torch
    gen = torch.Generator(device=device).manual_seed(int(seed))
    x = torch.randn(n_t, dtype=torch.float64, device=device, generator=gen)
    if pulsars:
        t = torch.arange(n_t, dtype=torch.float64, device=device) * tsamp
        for p in pulsars:
            cyc = p.f * t + 0.5 * p.fdot * t * t
            for h, (a, ph) in enumerate(zip(p.amps, p.phases), start=1):
                if a == 0.0:
                    continue
                ch = h * cyc
                ch = ch - torch.floor(ch)
                x += a * torch.cos(2.0 * math.pi * ch + ph)
        del t
    X = chirp_z_dft_head(x, n_t // 2) if any_length else torch.fft.rfft(x)[: n_t // 2]
    del x
    X[0] = 0.0
    med = torch.median(X[1:].real ** 2 + X[1:].imag ** 2)
    return (X / torch.sqrt(med / math.log(2.0))).to(torch.complex64)


def config5_device(device, trial: int = 0):
    """The wide workload generated on the device: 2^24 samples at 64 us and 16
    pulsars drawn as in config5 (a different noise realisation, drawn by
    torch from a seed of the same generator).  Returns (spectrum tensor,
    Spectrum with spec=None)."""
    c = CONFIGS[5]
    n_t, tsamp = c["n_t"], c["tsamp"]
    T = n_t * tsamp
    g = rng(5, 1000 + trial)
    ps = [draw_pulsar(g, T, tsamp, p_range=(1e-3, 20e-3), z_range=(-180.0, 180.0),
                      n_t=n_t) for _ in range(16)]
    X = _device_spectrum(n_t, tsamp, ps, int(g.integers(0, 2 ** 62)), device)
    return X, Spectrum(None, n_t, tsamp, ps)


def config2_device(device, trial: int = 0):
    """A single-DM trial generated on the device (the config2 recipe, a
    different realisation: pulsar drawn from generator (2, 1000 + trial),
    noise by torch from a seed of it).  Returns (spectrum tensor, Spectrum
    with spec=None)."""
    c = CONFIGS[2]
    n_t, tsamp = c["n_t"], c["tsamp"]
    T = n_t * tsamp
    g = rng(2, 1000 + trial)
    p = draw_pulsar(g, T, tsamp, n_t=n_t)
    X = _device_spectrum(n_t, tsamp, [p], int(g.integers(0, 2 ** 62)), device)
    return X, Spectrum(None, n_t, tsamp, [p])


def config3(device, trial: int = 0, n_spec: int | None = None):
    """Batched dedispersion trials, generated on the device (torch, FP64).

    n_spec spectra (256 by default) with series lengths log-uniform in
    [2^20, 2^23] samples (rounded to an even count), a sampling time drawn
    from 64 / 128 / 256 / 512 us, Gaussian noise, and in 10 % of them one
    binary pulsar drawn as in the single-DM workload.  Each series goes
    through the same recipe as to_spectrum (DFT, Nyquist dropped, DC zeroed,
    median normalisation), here with torch on the device so that 4.7e8 bins
    take seconds; the DFT of each length by chirp_z_dft_head, since an FFT
    library builds (and may compile) a plan for every distinct length.
    Returns (packed complex64 tensor, list of Trial).
    """
    import torch
    c = CONFIGS[3]
    g = rng(3, trial)
    n = c["n_spec"] if n_spec is None else int(n_spec)
    # log-uniform lengths, each rounded to an even sample count (n_t / 2 bins)
    want = np.exp(g.uniform(math.log(c["n_t_min"]), math.log(c["n_t_max"]), n))
    n_ts = np.clip(2 * np.rint(want / 2), c["n_t_min"], c["n_t_max"]).astype(np.int64)
    tsamps = g.choice(np.array(c["tsamps"]), size=n)
    with_psr = g.permutation(n)[: int(round(c["frac_pulsar"] * n))]
    seeds = g.integers(0, 2 ** 62, size=n)
    parts, trials, off = [], [], 0
    for i in range(n):
        n_t, tsamp = int(n_ts[i]), float(tsamps[i])
        psr = draw_pulsar(g, n_t * tsamp, tsamp, n_t=n_t) if i in with_psr else None
        X = _device_spectrum(n_t, tsamp, [psr] if psr else [], int(seeds[i]), device, any_length=True)
        parts.append(X)
        trials.append(Trial(off, n_t // 2, n_t, tsamp, psr))
        off += n_t // 2
    return torch.cat(parts), trials
