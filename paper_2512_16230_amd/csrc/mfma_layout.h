// Layout of the MFMA Hermite transform shared by the host (which builds the
// operand tables of a solve) and the step kernel that reads them.
//
// In lattice units the rows of order <= 3 are spanned by the 20 monomials of
// degree <= 3 of the integer velocity e_j, ordered
//   1, e_x, e_y, e_z, e_x^2, e_y^2, e_z^2, e_x e_y, e_x e_z, e_y e_z,
//   e_x^3, e_y^3, e_z^3, e_x e_y^2, e_x e_z^2, e_y e_x^2, e_y e_z^2,
//   e_z e_x^2, e_z e_y^2, e_x e_y e_z.
// The forward transform is the product of the monomial matrix (20 x b,
// padded to 32 x 64, scaled by the population's storage scale) with the
// stored numbers of 64 nodes; the back-transform is the product of the
// transposed monomial matrix (64 x 32, scaled by the output weight w_j of
// the population) with the 20 monomial coefficients of each node.  Both run
// as v_mfma_f32_32x32x16 products (f16 forward, bf16 backward) with FP32
// accumulation; each 16-byte table entry is one lane's A operand:
//   forward   [part (hi, lo)][k-step 0..3][lane]  A[row = lane % 32][K = 16 k + 8 (lane / 32) + t], t < 8
//   backward  [part (hi, lo)][m-block 0..1][k-step 0..1][lane]
//             A[row = 32 m + lane % 32][K = 16 k + 8 (lane / 32) + t]
// with K = population index (forward) or monomial index (backward).
#pragma once

namespace mrtlb {

constexpr int kMono = 20;                         // monomials of degree <= 3 in 3D
constexpr int kMfmaFwdVec = 2 * 4 * 64;           // 16-byte entries of the forward table
constexpr int kMfmaBwdVec = 2 * 2 * 2 * 64;       // and of the backward table
constexpr int kMfmaTabVec = kMfmaFwdVec + kMfmaBwdVec;
constexpr int kMfmaTabBytes = kMfmaTabVec * 16;   // 16 KB per solve

// Monomial P of the integer velocity (x, y, z).
__host__ __device__ constexpr int mono(int P, int x, int y, int z) {
  switch (P) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x;
    case 5: return y * y;
    case 6: return z * z;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return x * x * x;
    case 11: return y * y * y;
    case 12: return z * z * z;
    case 13: return x * y * y;
    case 14: return x * z * z;
    case 15: return y * x * x;
    case 16: return y * z * z;
    case 17: return z * x * x;
    case 18: return z * y * y;
    case 19: return x * y * z;
  }
  return 0;
}

}  // namespace mrtlb
