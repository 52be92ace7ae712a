// Matrix-core formulation of the length-4096 segment transforms (BF16 form).
//
// L = 4096 = 16 x 16 x 16, time n = 256 n1 + 16 n2 + n3, frequency
// k = k1 + 16 k2 + 256 k3 (all digits < 16).  With e(x) = exp(2 pi i x / 4096),
//   n k = 256 n1 k1 + 16 n2 k1 + n3 k1 + 256 n2 k2 + 16 n3 k2 + 256 n3 k3  (mod 4096),
// so the inverse transform y[n] = sum_k Y[k] e(n k) is three 16-point DFT
// stages whose twiddles all fold into the stage operators:
//   I1 (over k3, group k1):  A[n3][k3] = e(256 n3 k3 + n3 k1)     row scaling
//   I2 (over k2, group n3):  A[n2][k2] = e(256 n2 k2 + 16 n3 k2)  K scaling
//   I3 (over k1, group n2):  A[n1][k1] = e(256 n1 k1 + 16 n2 k1)  K scaling
// (n3 k1 depends on neither k2 nor n2, so it may be applied right after I1;
// 16 n2 k1 does not depend on n3, so it may wait until I3.)  The forward
// transform is the conjugate product in reverse order:
//   F1 (over n1, group n2):  A[k1][n1] = e(-256 k1 n1 - 16 n2 k1)  row scaling
//   F2 (over n2, group n3):  A[k2][n2] = e(-256 k2 n2 - 16 n3 k2)  row scaling
//   F3 (over n3, group k1):  A[k3][n3] = e(-256 k3 n3 - n3 k1)     K scaling
// Every group of 16 MFMA columns shares its group digit, so each group uses
// one operator and no twiddle is applied on the vector ALU.  A stage is one
// real 16x16x32 bf16 MFMA pair per group (the complex operator split into its
// real-output and imaginary-output rows), inputs bf16, accumulation FP32.
//
// Operand layout of v_mfma_f32_16x16x32_bf16 (lane l, c = l & 15, g = l >> 4):
//   A[i][k]: i = c, k = 8 g + e     B[k][j]: j = c, k = 8 g + e     D[i][j]: j = c, i = 4 g + e
// with K slot 8 g + 2 p + part holding part (re / im) of complex input 4 g + p.
//
// Groups and columns per stage (group Q < 16, column c = lane & 15):
//   stage k3 (I1 / F3): k1 = Q, column c -> k2 = c
//   stage k2 (I2 / F2): n3 = Q, column c -> k1 = c
//   stage k1 (I3 / F1): n2 = Q, column c -> n3 = c
//
// The forward stages exchange through two LDS buffers (one bf16 complex per
// 32-bit word) with additive layouts, so that every access is a per-lane base
// plus an immediate offset; the strides keep each access pattern free of bank
// conflicts (32 banks of 4 bytes), with one 128-bit side per transpose (the
// inverse stages use the chunk layout of correlate_m4k.hip instead):
//   buffer A ("x-contiguous"):  k1 * 324 + x + 20 * n3   (stage 2 reads 4 x in one b128)
//   buffer B ("k1-contiguous"): k1 + 324 * x + 20 * n3   (stage 3 reads 4 k1 in one b128)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdas {
namespace m4k {

constexpr int kL = 4096;
constexpr int kBufWords = 5184;   // last index 15*324 + 15 + 15*20 = 5175, rounded up

__host__ __device__ constexpr int addrA(int k1, int x, int n3) { return k1 * 324 + x + 20 * n3; }
__host__ __device__ constexpr int addrB(int k1, int x, int n3) { return k1 + 324 * x + 20 * n3; }

// Operator table: 1 op = 64 lanes x 4 words; each family is [group < 16][re rows, im rows].
constexpr int kOpWords = 256;
constexpr int OP_I1 = 0;      // inverse stage 1 (group k1)
constexpr int OP_I23 = 32;    // inverse stages 2 (group n3) and 3 (group n2): same operator
constexpr int OP_F12 = 64;    // forward stages 1 (group n2) and 2 (group n3): same operator
constexpr int OP_F3 = 96;     // forward stage 3 (group k1)
constexpr int kNumOps = 128;
constexpr size_t kTableBytes = (size_t)kNumOps * kOpWords * 4;

// Exponent (units of 1/4096 turn) of operator family `op0` for group G,
// output row `row` and input `pin`.
__host__ __device__ constexpr int64_t op_exponent(int op0, int G, int row, int pin) {
    return op0 == OP_I1    ? 256LL * row * pin + (int64_t)row * G
           : op0 == OP_I23 ? 256LL * row * pin + 16LL * G * pin
           : op0 == OP_F12 ? -(256LL * row * pin + 16LL * G * row)
                           : -(256LL * row * pin + (int64_t)pin * G);
}

// Bank order of template j: [j][Q][lane][p] bf16 pairs of H[Q + 16 (lane & 15) + 256 (4 (lane >> 4) + p)].
__host__ __device__ constexpr int bank_pos_of(int k) {
    return ((k & 15) * 64 + (((k >> 4) & 15) + 16 * ((k >> 8) >> 2))) * 4 + ((k >> 8) & 3);
}

}  // namespace m4k
}  // namespace fdas
