// Internal declarations shared by the libfdas translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/fdas.h"

namespace fdas {

constexpr int kPointsPerThread = 16;   // complex points each thread keeps in registers
constexpr int kMinLog2L = 10;
constexpr int kMaxLog2L = 14;

}  // namespace fdas

struct fdas_plan_s {
    fdas_config cfg;
    int32_t L = 0, log2L = 0, M = 0, V = 0;
    int32_t z_chunk = 0, n_chunks = 0;
    int32_t bank_elem = 0;       // bytes per complex template value
    int32_t tw_elem = 0;         // bytes per complex twiddle
    size_t ws_bytes = 0;
    size_t off_bank = 0, sz_bank = 0;
    size_t off_tw = 0, sz_tw = 0;
    size_t off_taps = 0, sz_taps = 0;      // FP64 taps, n_z x M complex (template build)
    size_t off_scr = 0, sz_scr = 0;        // peak counters
    size_t off_tab = 0, sz_tab = 0;        // matrix-core operator/twiddle tables
    bool mfma = false;                     // matrix-core correlation kernel (L = 4096 or 8192)
    int64_t peak_tile_cap = 0;             // number of peak tiles the scratch holds
    void *ws = nullptr;
    size_t ws_size = 0;
    bool templates_ready = false;
};

namespace fdas {

// Template bank + twiddle table (templates.hip).
hipError_t launch_make_templates(const fdas_plan_s &p, hipStream_t s);

// Matrix-core correlation, L = 8192, BF16 form (correlate_mfma.hip).
hipError_t launch_correlate_mfma(const fdas_plan_s &p, const void *spec, int64_t n,
                                 void *plane, hipStream_t s);

// Matrix-core correlation, L = 4096, BF16 form (correlate_m4k.hip).
hipError_t launch_correlate_m4k(const fdas_plan_s &p, const void *spec, int64_t n,
                                void *plane, hipStream_t s);

// Correlation (correlate.hip).
hipError_t launch_correlate(const fdas_plan_s &p, const void *spec, int64_t n,
                            void *plane, hipStream_t s);

// Peaks (peaks.hip).
constexpr int kPeakTileCols = 1024;   // columns per peak tile (one row per tile)
size_t peak_scratch_bytes(int64_t n_tiles);
hipError_t launch_peaks(const fdas_plan_s &p, const void *plane, int64_t n, float thr,
                        fdas_peak *out, int64_t capacity, int64_t *n_found, hipStream_t s);

}  // namespace fdas
