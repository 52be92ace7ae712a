// Matrix-core formulation of the length-4096 segment transforms (BF16 form).
//
// L = 4096 = 16 x 16 x 16, time n = 256 n1 + 16 n2 + n3, frequency
// k = k1 + 16 k2 + 256 k3 (all digits < 16).  Expanding n k mod 4096 gives,
// with W_N = exp(+2 pi i / N),
//   y[n] = sum_k1 W16^{n1 k1} T2(k1; n2, n3) sum_k2 W16^{n2 k2} T1(k2; n3)
//          sum_k3 W16^{n3 k3} Y[k1, k2, k3],
//   T1 = exp(2 pi i n3 k2 / 256),  T2 = exp(2 pi i (16 n2 + n3) k1 / 4096),
// and the forward transform is the conjugate product in reverse order.  All
// three stages are 16-point DFTs: one real 16x16x32 bf16 MFMA pair per group
// of 16 columns.  T1 depends on the stage-2 K index and on n3, shared by the
// group's columns, so it is folded into that stage's operator; T2 varies per
// column and is applied on the vector ALU between stages 2 and 3.
//
// Operand layout of v_mfma_f32_16x16x32_bf16 (lane l, c = l & 15, g = l >> 4):
//   A[i][k]: i = c, k = 8 g + e     B[k][j]: j = c, k = 8 g + e     D[i][j]: j = c, i = 4 g + e
// with K slot 8 g + 2 p + part holding part (re / im) of complex input 4 g + p.
//
// Work split: 8 waves per workgroup, wave w owns MFMA groups Q = 2 w + q (q < 2):
//   stage k3 (I1 / F3): k1 = Q, column c -> k2 = c
//   stage k2 (I2 / F2): n3 = Q, column c -> k1 = c
//   stage k1 (I3 / F1): n2 = Q, column c -> n3 = c
//
// LDS stage buffers (one bf16 complex per 32-bit word) use additive layouts so
// that every access is a per-lane base plus an immediate offset; the strides
// make each access pattern free of bank conflicts (32 banks of 4 bytes), with
// one 128-bit side per transpose:
//   buffer A ("x-contiguous"):  k1 * 324 + x + 20 * n3   (stage-2 reads 4 x in one b128)
//   buffer B ("k1-contiguous"): k1 + 324 * x + 20 * n3   (stage-3 reads 4 k1 in one b128)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdas {
namespace m4k {

constexpr int kL = 4096;
constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kBufWords = 5184;   // last index 15*324 + 15 + 15*20 = 5175, rounded up

__host__ __device__ constexpr int addrA(int k1, int x, int n3) { return k1 * 324 + x + 20 * n3; }
__host__ __device__ constexpr int addrB(int k1, int x, int n3) { return k1 + 324 * x + 20 * n3; }

// Operator table: 1 op = 64 lanes x 4 words.
constexpr int kOpWords = 256;
constexpr int OP_A16P = 0;    // 2: inverse DFT16 (re rows, im rows)
constexpr int OP_A2P = 2;     // 32: [n3][re/im] inverse DFT16 with T1 folded
constexpr int OP_A16M = 34;   // 2: forward DFT16
constexpr int OP_AF2M = 36;   // 32: [n3][re/im] forward DFT16 with conj(T1) folded
constexpr int kNumOps = 68;
// Per-lane twiddles (float2) after the operators:
//   inverse T2 [wave][lane][q < 2][e < 4];  forward conj(T2) [wave][lane][q < 2][e < 4]
constexpr int kT2Count = kWaves * 64 * 8;
constexpr size_t kTableBytes = (size_t)kNumOps * kOpWords * 4 + (size_t)2 * kT2Count * 8;

// Bank order of template j: [j][Q][lane][p] bf16 pairs of H[Q + 16 (lane & 15) + 256 (4 (lane >> 4) + p)].
__host__ __device__ constexpr int bank_pos_of(int k) {
    return ((k & 15) * 64 + (((k >> 4) & 15) + 16 * ((k >> 8) >> 2))) * 4 + ((k >> 8) & 3);
}

}  // namespace m4k
}  // namespace fdas
