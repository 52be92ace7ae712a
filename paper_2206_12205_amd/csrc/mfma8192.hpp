// Matrix-core (MFMA) formulation of the length-8192 segment transforms used
// by the BF16 precision form.
//
// Factorisation L = 8192 = 32 x 16 x 16 with time index
//   n = 256 n1 + 16 n2 + n3   (n1 < 32, n2 < 16, n3 < 16)
// and frequency index
//   k = k1 + 32 k2 + 512 k3   (k1 < 32, k2 < 16, k3 < 16).
// Expanding n k mod 8192 gives, with W_N = exp(+2 pi i / N),
//   y[n] = sum_k1 W32^{n1 k1} T2(k1; n2, n3) sum_k2 W16^{n2 k2} T1(k2; n3)
//          sum_k3 W16^{n3 k3} Y[k1, k2, k3],
//   T1 = exp(2 pi i n3 k2 / 256),  T2 = exp(2 pi i (16 n2 + n3) k1 / 8192).
// The forward transform is the same product with every factor conjugated and
// the stages run in the opposite order.
//
// Each stage is a batch of small DFTs, computed as real 16x16x32 bf16 MFMA
// products: a complex 16-point DFT acting on 16 columns is the real
// [[Re, -Im], [Im, Re]] operator, split in a "real rows" and an "imaginary
// rows" MFMA; a 32-point DFT uses 4 row blocks x 2 K blocks.  Stage inputs
// are bfloat16, accumulation is FP32 (the BF16 storage / FP32 accumulation
// form).  The twiddle T1 depends only on the stage-2 K index and on n3, which
// every column of a stage-2 MFMA shares, so it is folded into that stage's
// operator; T2 varies per column and is applied on the vector ALU.
//
// Operand layout of v_mfma_f32_16x16x32_bf16 (lane l, c = l & 15, g = l >> 4):
//   A[i][k]: i = c, k = 8 g + e (e < 8)     B[k][j]: j = c, k = 8 g + e
//   D[i][j]: j = c, i = 4 g + e (e < 4)
// K slots are paired (re, im) of one complex input: slot 8g + 2p + part holds
// part (0 = re, 1 = im) of complex input 4g + p (p < 4).
//
// Work split of one workgroup (8 waves, wave w) over the 512/512/256 stage
// instances, 16 columns per MFMA group:
//   stage k3 (I1 / F3): group Q = 4w + q (q < 4): k1 = Q, column c -> k2 = c
//   stage k2 (I2 / F2): group Q = 4w + q: n3 = 4 (w % 4) + q, c -> k1 = 16 (w / 4) + c
//   stage k1 (I3 / F1): group Q = 2w + q (q < 2): n2 = Q, c -> n3 = c
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdas {
namespace m8k {

constexpr int kL = 8192;
constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;

// LDS word address (one bf16 complex per 32-bit word) of element (k1, x, n3)
// of a [32][16][16] stage buffer, XOR-swizzled against bank conflicts of the
// four transpose access patterns.
__host__ __device__ constexpr int lds_addr(int k1, int x, int n3) {
    return k1 * 256 + ((x * 16 + n3) ^ ((k1 * 4 + (x >> 1) * 9) & 31));
}

// Operand table in the workspace: 1 Op = 64 lanes x 4 words (1 KiB).
constexpr int kOpWords = 256;
constexpr int OP_A16P = 0;     // 2 ops: inverse DFT16 (re rows, im rows)
constexpr int OP_A2P = 2;      // 32 ops: [n3][re/im] inverse DFT16 with T1 folded
constexpr int OP_A32P = 34;    // 8 ops: [mb][kb] inverse DFT32
constexpr int OP_A32M = 42;    // 8 ops: [mb][kb] forward DFT32
constexpr int OP_AF2M = 50;    // 32 ops: [n3][re/im] forward DFT16 with conj(T1) folded
constexpr int OP_A16M = 82;    // 2 ops: forward DFT16
constexpr int kNumOps = 84;
// Per-lane twiddles (float2), after the operators:
//   inverse T2: [wave][lane][q < 4][e < 4]
//   forward conj(T2): [wave][lane][q < 2][mb < 4][e2 < 2]
constexpr int kT2Count = kWaves * 64 * 16;
constexpr int kT2FCount = kWaves * 64 * 16;
constexpr size_t kTableBytes = (size_t)kNumOps * kOpWords * 4 + (size_t)(kT2Count + kT2FCount) * 8;

// Bank layout of template j: [j][wave][q < 4][lane][p < 4] bf16 pairs holding
// H[k1 + 32 k2 + 512 k3] with k1 = 4 wave + q, k2 = c, k3 = 4 g + p.
__host__ __device__ constexpr int bank_freq_index(int wave, int q, int lane, int p) {
    return (4 * wave + q) + 32 * (lane & 15) + 512 * (4 * (lane >> 4) + p);
}

}  // namespace m8k
}  // namespace fdas
