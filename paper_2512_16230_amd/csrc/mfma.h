// Step kernel with the Hermite transforms on the matrix cores (MFMA), for the
// 3D lattices (|e| <= 2) with int16 deviation storage: the same update as
// k_step (a1-a8), with a3 and a7 as dense products.
//
// A wavefront handles 64 consecutive nodes of one row.  Each lane gathers
// the b populations of its own node (a1, as k_step) and parks them in LDS;
// the forward transform (a3) then reads them as the B operand of
// v_mfma_f32_32x32x16_f16, two groups of 32 nodes per wavefront:
//   R = E f_lo + 2E f_hi - 99328 E 1,   E = monomials x storage scale / sigma,
// where each int16 number q enters exactly as two f16 numbers whose bits
// are the bits of q, rearranged (one or two integer instructions per pair of
// numbers): f_lo = 1024 + (q mod 1024) and f_hi = 2^15 + 512 k' with
// k' = q div 1024 + 32, so that q = f_lo + 2 f_hi - 99328; E is split into two
// f16 parts (2E is exact too), so the products are exact and only the FP32
// accumulation rounds.  A lane-half swap (v_permlane32_swap) gives every lane the 20
// monomial sums of its own node; moment space (a2, a4-a6) runs per node as in
// k_step and yields the 20 monomial coefficients C of the back-transform
// (a7), which run, split into bf16 hi + lo, through
// v_mfma_f32_32x32x16_bf16 against the transposed monomial matrix scaled by
// the output weights (bf16 hi + lo; three products, lo x lo dropped).  The
// outputs meet the stored numbers again in LDS, become int16 there and are
// stored by their own lanes (a8, as k_step).
#pragma once

#include "device.h"
#include "mfma_layout.h"

namespace mrtlb {

typedef _Float16 mfma_h8 __attribute__((ext_vector_type(8)));
typedef __bf16 mfma_b8 __attribute__((ext_vector_type(8)));
typedef float mfma_f16x __attribute__((ext_vector_type(16)));
typedef uint32_t mfma_u4 __attribute__((ext_vector_type(4)));
typedef uint32_t mfma_u2 __attribute__((ext_vector_type(2)));

// LDS staging of one wavefront: per node 64 int16 slots (32 dwords) plus two
// dwords of padding, so 8-byte rows of consecutive nodes start in different
// banks.
constexpr int kStageStride = 34;

// Forward operand chunks of two packed int16 numbers q (one per half), as
// f16 bits: lo = 1024 + (q & 1023) (exponent 10, the low ten bits of q as the
// significand), hi = 2^15 (1 + k' / 64) with k' the six high bits of q with
// the sign bit flipped (exponent 15, k' in the top six significand bits).
// `one` holds 0x64006400 in a register (keeps the or of the low chunk in one
// instruction).
__device__ __forceinline__ uint32_t chunk_lo(uint32_t q2, uint32_t one) { return (q2 & 0x03FF03FFu) | one; }
__device__ __forceinline__ uint32_t chunk_hi(uint32_t q2) {
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  const u16x2 sh = __builtin_bit_cast(u16x2, q2) >> (u16x2){6, 6};
  return __builtin_amdgcn_bitop3_b32(__builtin_bit_cast(uint32_t, sh), 0x03F003F0u, 0x7A007A00u, 0x6A);
}

// Two floats as packed bf16 (round to nearest even) and the floats they stand for.
typedef float mfma_f2 __attribute__((ext_vector_type(2)));
typedef __bf16 mfma_bf2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16x2_bits(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((mfma_f2){a, b}, mfma_bf2));
}
__device__ __forceinline__ float bf16_lo_value(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ float bf16_hi_value(uint32_t h) { return __uint_as_float(h & 0xFFFF0000u); }

__device__ __forceinline__ float swap_lo(float x, float y, float& hi_out) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  hi_out = __uint_as_float(r[1]);
  return __uint_as_float(r[0]);
}

template <class L, int MODEL>
__global__ __launch_bounds__(kBlock) void k_step_mfma(const Job<float>* __restrict__ jobs, int njobs,
                                                     uint32_t total_blocks) {
  constexpr int ST = kI16Dev;
  using Real = float;
  using T = int16_t;
  constexpr int B = L::B;
  static_assert(L::D == 3 && B <= 64 && L::MAXE <= 2, "MFMA transform: 3D lattices with |e| <= 2");
  __shared__ mfma_u4 tab[kMfmaTabVec];
  __shared__ uint32_t stage[kBlock / 64][64 * kStageStride];

  const uint32_t lin = xcd_remap(blockIdx.x, total_blocks);
  const int jb = njobs > 1 ? find_job(jobs, njobs, lin) : 0;
  const Job<Real>& J = jobs[jb];
  const KParams<Real>& P = J.P;
  {
    const mfma_u4* gt = static_cast<const mfma_u4*>(J.mtab);
    for (int k = threadIdx.x; k < kMfmaTabVec; k += kBlock) tab[k] = gt[k];
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int h = lane >> 5, il = lane & 31;
  uint32_t* sq = stage[threadIdx.x >> 6];
  int ix, iy, iz;
  // a wavefront covers 64 slots of one row (the row pitch is a multiple of 64)
  const bool valid = tile_node<1>(J, lin - J.block_begin, ix, iy, iz);
  if (__all(!valid)) return;
  RowGeom<L> g;
  g.init(iy, iz, P.nx, P.nxp, P.ny, P.nz);

  // a1: gather the own node, park the stored numbers in LDS (slot = population)
  {
    T raw[B][1];
    if (valid) {
      gather<L, ST, 1, false>(J, g, ix, raw);
    } else {
      static_for<0, B>([&](auto jj) { raw[decltype(jj)::value][0] = 0; });
    }
    static_for<0, 32>([&](auto pp) {
      constexpr int p = decltype(pp)::value;
      const uint32_t a = 2 * p < B ? (uint16_t)raw[2 * p < B ? 2 * p : 0][0] : 0u;
      const uint32_t b = 2 * p + 1 < B ? (uint16_t)raw[2 * p + 1 < B ? 2 * p + 1 : 0][0] : 0u;
      sq[lane * kStageStride + p] = a | (b << 16);
    });
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // a3: forward products, group gr = nodes 32 gr .. 32 gr + 31 of the wavefront
  mfma_f16x acc[2] = {mfma_f16x{}, mfma_f16x{}};
  uint32_t one = 0x64006400u;
  asm volatile("" : "+v"(one));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const mfma_h8 ahi = __builtin_bit_cast(mfma_h8, tab[(0 * 4 + k) * 64 + lane]);
    const mfma_h8 alo = __builtin_bit_cast(mfma_h8, tab[(1 * 4 + k) * 64 + lane]);
    const mfma_h8 ahi2 = ahi + ahi, alo2 = alo + alo;   // exact in f16
#pragma unroll
    for (int gr = 0; gr < 2; ++gr) {
      const uint32_t* src = sq + (32 * gr + il) * kStageStride + 8 * k + 4 * h;
      const mfma_u2 q01 = *reinterpret_cast<const mfma_u2*>(src);
      const mfma_u2 q23 = *reinterpret_cast<const mfma_u2*>(src + 2);
      const mfma_u4 lo = {chunk_lo(q01[0], one), chunk_lo(q01[1], one), chunk_lo(q23[0], one), chunk_lo(q23[1], one)};
      const mfma_u4 hi = {chunk_hi(q01[0]), chunk_hi(q01[1]), chunk_hi(q23[0]), chunk_hi(q23[1])};
      const mfma_h8 blo = __builtin_bit_cast(mfma_h8, lo);
      const mfma_h8 bhi = __builtin_bit_cast(mfma_h8, hi);
      acc[gr] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, blo, acc[gr], 0, 0, 0);
      acc[gr] = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo, blo, acc[gr], 0, 0, 0);
      acc[gr] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi2, bhi, acc[gr], 0, 0, 0);
      acc[gr] = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo2, bhi, acc[gr], 0, 0, 0);
    }
  }

  // every lane takes the 20 monomial sums of its own node (node = lane):
  // register r of group gr holds row 8 (r / 4) + 4 h + r % 4 of node 32 gr + il
  Real R[kMono];
#pragma unroll
  for (int r = 0; r < 12; ++r) {
    float up;
    const float low = swap_lo(acc[0][r], acc[1][r], up);
    const int row0 = 8 * (r / 4) + r % 4;
    R[row0] = P.msig * (low - P.mbias[row0]);
    if (row0 + 4 < kMono) R[row0 + 4] = P.msig * (up - P.mbias[row0 + 4]);
  }

  // a2, a4-a6 in moment space, per node
  Moments<Real> Mo;
  {
    const Real R1[3] = {R[1], R[2], R[3]}, R2n[3] = {R[4], R[5], R[6]}, R2o[3] = {R[7], R[8], R[9]};
    const Real R3p[3] = {R[10], R[11], R[12]};
    const Real R3m[3][3] = {{0, R[13], R[14]}, {R[15], 0, R[16]}, {R[17], R[18], 0}};
    finish_moments<3, is_standard<L>()>(P, R[0], R1, R2n, R2o, R3p, R3m, R[19], Mo);
  }
  Targets<Real> Tg;
  relax_node<L, ST, MODEL, false>(Mo, J, g, valid ? ix : 0, Tg);
  BackCoeffs<Real> C;
  back_coeffs<3, is_standard<L>()>(P, Tg.d0, Tg.d1, Tg.d2n, Tg.d2o, Tg.d3m, Tg.d3p, Tg.dxyz, C);
  const Real c[kMono] = {C.b0,     C.b1[0],     C.b1[1],     C.b1[2],     C.b2n[0],    C.b2n[1],   C.b2n[2],
                         C.b2o[0], C.b2o[1],    C.b2o[2],    C.b3p[0],    C.b3p[1],    C.b3p[2],   C.b3m[0][1],
                         C.b3m[0][2], C.b3m[1][0], C.b3m[1][2], C.b3m[2][0], C.b3m[2][1], C.bxyz};

  // B operands of the back-transform: monomial K of node 32 gr + il sits in
  // lane half (K / 8) % 2 of k-step K / 16; the own node's coefficients are
  // split into bf16 hi + lo and swapped into place
  uint32_t opA[2][2][4], opB[2][2][4];   // [part][k-step][dword]
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      uint32_t v0[2], v1[2];   // [part] for the slots of half 0 and half 1
      const int K0 = 16 * k + 2 * d, K1 = 16 * k + 8 + 2 * d;
      auto split = [&](int K, uint32_t (&out)[2]) {
        const float a = K < kMono ? c[K < kMono ? K : 0] : 0.0f;
        const float b = K + 1 < kMono ? c[K + 1 < kMono ? K + 1 : 0] : 0.0f;
        out[0] = bf16x2_bits(a, b);
        out[1] = bf16x2_bits(a - bf16_lo_value(out[0]), b - bf16_hi_value(out[0]));
      };
      split(K0, v0);
      split(K1, v1);
#pragma unroll
      for (int part = 0; part < 2; ++part) {
        const auto r = __builtin_amdgcn_permlane32_swap(v0[part], v1[part], false, false);
        opA[part][k][d] = r[0];
        opB[part][k][d] = r[1];
      }
    }

  // a7: back-transform and the output numbers, group by group in LDS:
  // o_j = kin (1 - s_h) q_j + sum_P w_j e_j^P C_P (row j = population)
  const Real kxe = Tg.kx * P.kin;
  float smax = 0.0f;
#pragma unroll
  for (int gr = 0; gr < 2; ++gr) {
    const int node = 32 * gr + il;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      mfma_f16x out = {};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const mfma_b8 ahi = __builtin_bit_cast(mfma_b8, tab[kMfmaFwdVec + ((0 * 2 + m) * 2 + k) * 64 + lane]);
        const mfma_b8 alo = __builtin_bit_cast(mfma_b8, tab[kMfmaFwdVec + ((1 * 2 + m) * 2 + k) * 64 + lane]);
        const uint32_t(&bh)[4] = gr == 0 ? opA[0][k] : opB[0][k];
        const uint32_t(&bl)[4] = gr == 0 ? opA[1][k] : opB[1][k];
        const mfma_b8 bhi = __builtin_bit_cast(mfma_b8, mfma_u4{bh[0], bh[1], bh[2], bh[3]});
        const mfma_b8 blo = __builtin_bit_cast(mfma_b8, mfma_u4{bl[0], bl[1], bl[2], bl[3]});
        out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi, out, 0, 0, 0);
        out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo, out, 0, 0, 0);
        out = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi, out, 0, 0, 0);
      }
      // register 4 qd + u holds population 32 m + 8 qd + 4 h + u of the node
#pragma unroll
      for (int qd = 0; qd < 4; ++qd) {
        if (32 * m + 8 * qd >= B) continue;   // padding rows only
        uint32_t* dst = sq + node * kStageStride + 16 * m + 4 * qd + 2 * h;
        const mfma_u2 q = *reinterpret_cast<const mfma_u2*>(dst);
        float o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int16_t qv = (int16_t)((q[u >> 1] >> (16 * (u & 1))) & 0xFFFFu);
          o[u] = kxe * (float)qv + out[4 * qd + u];
        }
        smax = __builtin_fmaxf(smax, __builtin_fmaxf(__builtin_fmaxf(fabsf(o[0]), fabsf(o[1])),
                                                     __builtin_fmaxf(fabsf(o[2]), fabsf(o[3]))));
        const mrtlb_short2 p01 = snorm16x2(o[0], o[1]);
        const mrtlb_short2 p23 = snorm16x2(o[2], o[3]);
        *reinterpret_cast<mfma_u2*>(dst) = mfma_u2{__builtin_bit_cast(uint32_t, p01), __builtin_bit_cast(uint32_t, p23)};
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // int16: a conversion clamped at +-1 flags the solve
  if (smax > 1.0f) *J.sat = 1;
  if (!valid) return;

  // a8: the own node's output numbers from LDS to HBM
  T outv[B][1];
  static_for<0, 32>([&](auto pp) {
    constexpr int p = decltype(pp)::value;
    if constexpr (2 * p < B) {
      const uint32_t v = sq[lane * kStageStride + p];
      outv[2 * p][0] = (T)(v & 0xFFFFu);
      if constexpr (2 * p + 1 < B) outv[2 * p + 1][0] = (T)(v >> 16);
    }
  });
  const auto rout = make_rsrc(J.fout, P.pop_bytes);
  const uint32_t lo = g.lown() + (uint32_t)ix;
  static_for<0, B>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    store_vec<ST, 1>(rout, (uint32_t)j * (uint32_t)P.nxp, lo, outv[j]);
  });
}

}  // namespace mrtlb
