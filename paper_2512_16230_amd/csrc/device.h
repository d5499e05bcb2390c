// Device code of the Hermite-matrix MRT lattice Boltzmann library: the
// fused pull collide-and-stream kernel and its helpers (initialisation,
// read-out, restore, FP64 plane sums), plus the host-side launchers that
// instantiate them for one lattice.  Included by one translation unit per
// lattice (inst_*.hip) so the instantiations compile in parallel.
//
// MI355X (gfx950) kernels and C ABI of the Hermite-matrix MRT lattice
// Boltzmann method (arXiv 2512.16230): fused pull collide-and-stream,
// initialisation, moment read-out, checkpoint and FP64 conserved sums.
//
// Layout in HBM: populations row-blocked (see RowGeom: every grid row holds
// its b population rows back to back, x fastest), two buffers (pull
// propagation, double-buffered).  The buffer holds the post-collision
// populations of the previous step, so f_bar_j(x, t) = buf_j(x - e_j): a
// step gathers along -e_j, collides in registers and writes every
// population at its own node (coalesced stores).
//
// Collision (per node, registers only).  With the component Hermite rows of
// order <= 3 (H0 = 1, H1 = c, H2 = cc - cs^2, H3 mixed / xyz / corrected
// pure) and every row above third order relaxing at the single rate s_h,
// the update of eq. (2-3) with Lambda = H^-1 S H is
//     f* = (1 - s_h) f + W sum_{r<=3} H_r (m*_r - (1 - s_h) m_r) / n_r
// (the reduced form of eq. H-MRT-LB-1).  The forward moments are taken as
// raw monomial sums over symmetric velocity pairs (even monomials from
// f_p + f_q, odd ones from f_p - f_q) and the back-transform as a monomial
// polynomial evaluated per pair, so each population costs a few FMAs and no
// b x b matrix is formed.  The normal second-order rows relax their trace at
// s_bulk and their deviator at s_shear.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "kernels.h"
#include "lattices.h"
#include "launch.h"

namespace mrtlb {

// ---------------------------------------------------------------------------
// compile-time helpers
// ---------------------------------------------------------------------------

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <class L>
constexpr int evel(int j, int a) {
  return a == 0 ? L::EX[j] : (a == 1 ? L::EY[j] : ez<L>(j));
}


__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// ---------------------------------------------------------------------------
// storage formats
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

template <int ST>
struct StoreT;
template <>
struct StoreT<kFP64> { using T = double; using Real = double; };
template <>
struct StoreT<kFP32> { using T = float; using Real = float; };
template <>
struct StoreT<kFP32Dev> { using T = float; using Real = float; };
template <>
struct StoreT<kFP32DevF64> { using T = float; using Real = double; };
template <>
struct StoreT<kFP16Dev> { using T = _Float16; using Real = float; };
template <>
struct StoreT<kBF16Dev> { using T = uint16_t; using Real = float; };
template <>
struct StoreT<kI16Dev> { using T = int16_t; using Real = float; };

// Global-address-space access with a 32-bit byte offset from a uniform base:
// the base stays in SGPRs and each lane supplies one 32-bit offset
// (global_load/store with saddr), instead of flat accesses with a 64-bit
// address per lane.  Every population plane is smaller than 4 GiB.
#define MRTLB_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ T gload(const void* base, uint32_t byteoff) {
  const MRTLB_GLOBAL char* p = (const MRTLB_GLOBAL char*)base;
  return *(const MRTLB_GLOBAL T*)(p + byteoff);
}

template <class T>
__device__ __forceinline__ void gstore(void* base, uint32_t byteoff, T v) {
  MRTLB_GLOBAL char* p = (MRTLB_GLOBAL char*)base;
  *(MRTLB_GLOBAL T*)(p + byteoff) = v;
}

// ---------------------------------------------------------------------------
// node geometry: wrapped row offsets for -MAXE..MAXE along y and z
// ---------------------------------------------------------------------------

// Population layout in HBM (row-blocked): element (j, x, y, z) of a buffer
// sits at ((r * b + j) * nxp + x) with node row r = z * ny + y and the row
// pitch nxp = nx rounded up to 32 nodes, i.e. every row of nx nodes stores
// its b population rows back to back, each starting on a 32-element boundary.  A step then
// reads each population from 2*MAXE+1 (2D) neighbouring row blocks and
// writes one row block, instead of touching b planes that lie a whole
// domain apart.  Scalar node fields (phi, force) are plain [r][x].
template <class L>
struct RowGeom {
  static constexpr int M = L::MAXE;
  uint32_t yo[2 * M + 1];   // wrap(iy - s)
  uint32_t zo[2 * M + 1];   // wrap(iz - s) * ny
  int nx, nxp;

  __device__ __forceinline__ void init(int iy, int iz, int nx_, int nxp_, int ny, int nz) {
    nx = nx_;
    nxp = nxp_;
#pragma unroll
    for (int s = -M; s <= M; ++s) {
      yo[s + M] = (uint32_t)wrap(iy - s, ny);
      if constexpr (L::D == 3) zo[s + M] = (uint32_t)wrap(iz - s, nz) * (uint32_t)ny;
    }
  }
  // node row of the source of population j (pull: row of x - e_j)
  template <int J>
  __device__ __forceinline__ uint32_t row() const {
    uint32_t r = yo[L::EY[J] + M];
    if constexpr (L::D == 3) r += zo[ez<L>(J) + M];
    return r;
  }
  __device__ __forceinline__ uint32_t own_row() const { return yo[M] + (L::D == 3 ? zo[M] : 0u); }
  // first element of population J's source row
  template <int J>
  __device__ __forceinline__ uint32_t prow() const { return (row<J>() * (uint32_t)L::B + J) * (uint32_t)nxp; }
  // first element of population j's own row
  __device__ __forceinline__ uint32_t pown(int j) const { return (own_row() * (uint32_t)L::B + j) * (uint32_t)nxp; }
  // The step kernel splits an element index into a wave-uniform part, added
  // to the buffer pointer in scalar registers, and a per-lane part that
  // depends on the source row only (plus, at the periodic x-edges, on e_x):
  //   source of population J (J >= 1):  uni = J nxp - e_Jx - M,
  //                                     lane = row_J b nxp + (x_src + e_Jx + M)
  //   own row:                          uni = J nxp, lane = own b nxp + x.
  // Both parts are non-negative (nxp >= 32 > 2M) and sum to the index.
  template <int J>
  __device__ __forceinline__ uint32_t lrow() const { return row<J>() * (uint32_t)L::B * (uint32_t)nxp; }
  __device__ __forceinline__ uint32_t lown() const { return own_row() * (uint32_t)L::B * (uint32_t)nxp; }
  template <int J>
  __device__ __forceinline__ uint32_t uni_src() const { return (uint32_t)(J * nxp - L::EX[J] - M); }
  // element of the source of population J for node ix (periodic in x)
  template <int J>
  __device__ __forceinline__ uint32_t src(int ix) const { return prow<J>() + (uint32_t)wrap(ix - L::EX[J], nx); }
  // node index (scalar fields) of the own node ix
  __device__ __forceinline__ uint32_t node(int ix) const { return own_row() * (uint32_t)nx + (uint32_t)ix; }
  // node index of the node ix shifted by s = +-1 along axis a
  __device__ __forceinline__ uint32_t shifted(int ix, int a, int s) const {
    uint32_t xi = (uint32_t)ix, yi = yo[M], zi = (L::D == 3 ? zo[M] : 0u);
    if (a == 0) xi = (uint32_t)wrap(ix + s, nx);
    if (a == 1) yi = yo[M - s];
    if constexpr (L::D == 3) {
      if (a == 2) zi = zo[M - s];
    }
    return (yi + zi) * (uint32_t)nx + xi;
  }
};

// Vectors of VEC consecutive stored elements.  Loads start at any element
// (alignment of one element: the pull shift), stores at own nodes are
// aligned to the whole vector.
template <class T, int VEC, int ALIGN>
struct VecT {
  typedef T type __attribute__((ext_vector_type(VEC), aligned(ALIGN)));
};

// Populations are streamed once per step: the step kernel's stores carry the
// nontemporal hint (MRTLB_NT=0 at build time turns it off).
#ifndef MRTLB_NT
#define MRTLB_NT 1
#endif

// The step kernel reads and writes population buffers through buffer
// resources (MUBUF): the base address lives in the resource, the wave-uniform
// part of an offset in soffset (SGPR) and each lane supplies one 32-bit byte
// offset, so per population no per-lane address arithmetic is needed.
// Accesses beyond the resource's size read 0 / are dropped.
constexpr int kBufFlags = 0x00020000;   // dword 3 of a raw buffer resource (gfx9 family)
// cache policy bits (gfx94x/gfx950 encoding: 1 = sc0, 2 = nt, 16 = sc1).
// Stores are streamed (nt) at device scope (sc1); loads keep the default
// policy: a wavefront's shifted read spans one partial cache line at each
// end, which the neighbouring wavefront reads from L2.  Measured on rD2Q25
// FP32: nontemporal loads 3-6% slower; nt stores without sc1 2% slower.
#ifndef MRTLB_LOAD_AUX
#define MRTLB_LOAD_AUX 0
#endif
#ifndef MRTLB_STORE_AUX
#define MRTLB_STORE_AUX (MRTLB_NT ? 18 : 0)
#endif
constexpr int kAuxLoad = MRTLB_LOAD_AUX;
constexpr int kAuxStore = MRTLB_STORE_AUX;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kBufFlags);
}

template <int BYTES>
struct RawChunk;
template <>
struct RawChunk<2> { using T = unsigned short; };
template <>
struct RawChunk<4> { using T = unsigned int; };
template <>
struct RawChunk<8> { typedef unsigned int T __attribute__((ext_vector_type(2))); };
template <>
struct RawChunk<16> { typedef unsigned int T __attribute__((ext_vector_type(4))); };

template <int BYTES>
__device__ __forceinline__ typename RawChunk<BYTES>::T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (BYTES == 2) return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, kAuxLoad);
  else if constexpr (BYTES == 4) return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, kAuxLoad);
  else if constexpr (BYTES == 8) return __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, kAuxLoad);
  else return __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, kAuxLoad);
}

template <int BYTES>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, typename RawChunk<BYTES>::T v, uint32_t voff,
                                          uint32_t soff) {
  if constexpr (BYTES == 2) __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)voff, (int)soff, kAuxStore);
  else if constexpr (BYTES == 4) __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, (int)soff, kAuxStore);
  else if constexpr (BYTES == 8) __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)voff, (int)soff, kAuxStore);
  else __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)voff, (int)soff, kAuxStore);
}

// VEC consecutive stored elements starting at element (uni + lane): uni is
// wave-uniform, lane per lane.  Loads start at any element (the pull shift);
// vectors wider than 16 bytes are split into 16-byte pieces.
template <int ST, int VEC>
__device__ __forceinline__ void load_vec(__amdgpu_buffer_rsrc_t r, uint32_t uni, uint32_t lane,
                                         typename StoreT<ST>::T (&out)[VEC]) {
  using T = typename StoreT<ST>::T;
  constexpr int BYTES = VEC * (int)sizeof(T);
  constexpr int PIECE = BYTES > 16 ? 16 : BYTES;
  constexpr int PER = PIECE / (int)sizeof(T);
#pragma unroll
  for (int c = 0; c < VEC / PER; ++c) {
    const auto v = buf_load<PIECE>(r, lane * (uint32_t)sizeof(T), (uni + (uint32_t)(c * PER)) * (uint32_t)sizeof(T));
    struct Elems { T e[PER]; };
    const Elems el = __builtin_bit_cast(Elems, v);
#pragma unroll
    for (int k = 0; k < PER; ++k) out[c * PER + k] = el.e[k];
  }
}

template <int ST, int VEC>
__device__ __forceinline__ void store_vec(__amdgpu_buffer_rsrc_t r, uint32_t uni, uint32_t lane,
                                          const typename StoreT<ST>::T (&in)[VEC]) {
  using T = typename StoreT<ST>::T;
  constexpr int BYTES = VEC * (int)sizeof(T);
  constexpr int PIECE = BYTES > 16 ? 16 : BYTES;
  constexpr int PER = PIECE / (int)sizeof(T);
#pragma unroll
  for (int c = 0; c < VEC / PER; ++c) {
    struct Elems { T e[PER]; };
    Elems el;
#pragma unroll
    for (int k = 0; k < PER; ++k) el.e[k] = in[c * PER + k];
    buf_store<PIECE>(r, __builtin_bit_cast(typename RawChunk<PIECE>::T, el), lane * (uint32_t)sizeof(T),
                     (uni + (uint32_t)(c * PER)) * (uint32_t)sizeof(T));
  }
}

// Storage conversions are never fused with neighbouring arithmetic: the
// scaled value is rounded to FP32 first, then RNE to the 16-bit format,
// whatever code shape the compiler picks for the surrounding kernel (LLVM
// otherwise turns fptrunc(fmul) into a single-rounding v_fma_mixlo_f16 in
// some unrollings and not in others).  pin() is an empty asm statement that
// makes its operand an opaque FP32 register value.
__device__ __forceinline__ float pin(float v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Storage with a per-population scale (the 16-bit deviation formats).
template <int ST>
constexpr bool scaled_storage() { return ST == kFP16Dev || ST == kBF16Dev || ST == kI16Dev; }

// The number a stored element reads as (before its scale).
template <int ST>
__device__ __forceinline__ typename StoreT<ST>::Real units(typename StoreT<ST>::T v) {
  using Real = typename StoreT<ST>::Real;
  if constexpr (ST == kFP16Dev) {
    return (float)v;
  } else if constexpr (ST == kBF16Dev) {
    return bf16_to_f32(v);
  } else if constexpr (ST == kI16Dev) {
    return (float)(int)v;
  } else {
    return (Real)v;
  }
}

// int16 fixed point: round(clamp(o, -1, 1) * 32767) to the nearest integer
// of the exact product, two values per instruction (v_cvt_pknorm_i16_f32).
typedef short mrtlb_short2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void snorm16x2(float a, float b, int16_t& qa, int16_t& qb) {
  const mrtlb_short2 r = __builtin_amdgcn_cvt_pknorm_i16(a, b);
  qa = r[0];
  qb = r[1];
}
__device__ __forceinline__ mrtlb_short2 snorm16x2(float a, float b) { return __builtin_amdgcn_cvt_pknorm_i16(a, b); }

// Output number -> stored element.  FP16/BF16 round the FP32 value to
// nearest even; int16 as snorm16x2.
template <int ST>
__device__ __forceinline__ typename StoreT<ST>::T to_stored(typename StoreT<ST>::Real o) {
  using T = typename StoreT<ST>::T;
  if constexpr (ST == kFP16Dev) {
    return (_Float16)pin(o);
  } else if constexpr (ST == kBF16Dev) {
    return f32_to_bf16_rne(o);
  } else if constexpr (ST == kI16Dev) {
    int16_t q, unused;
    snorm16x2(o, 0.0f, q, unused);
    return q;
  } else {
    return (T)o;
  }
}

template <int ST, class Real>
__device__ __forceinline__ Real decode(typename StoreT<ST>::T v, const KParams<Real>& P, int j) {
  if constexpr (scaled_storage<ST>()) {
    return (Real)pin(units<ST>(v) * (float)P.wsc[j]);
  } else {
    return (Real)v;
  }
}

template <int ST, class Real>
__device__ __forceinline__ typename StoreT<ST>::T encode(Real v, const KParams<Real>& P, int j) {
  using T = typename StoreT<ST>::T;
  if constexpr (scaled_storage<ST>()) {
    return to_stored<ST>(pin((float)v * (float)P.iwsc[j]));
  } else {
    return (T)v;
  }
}

// int16 storage: an output number beyond [-1, 1] saturates in the
// conversion.  Kernels that write int16 populations keep the largest
// |output number| and raise the solve's flag (a plain vector store of 1)
// when it exceeds 1; the host reports it at the next synchronous read.
template <int ST, class Real>
__device__ __forceinline__ float sat_of(Real v, const KParams<Real>& P, int j) {
  if constexpr (ST == kI16Dev) return fabsf((float)v * (float)P.iwsc[j]);
  else return 0.0f;
}

template <int ST, class Real>
__device__ __forceinline__ void raise_saturation(const Job<Real>& J, float smax) {
  if constexpr (ST == kI16Dev) {
    if (smax > 1.0f) *J.sat = 1;
  }
}

// int16 saturation: an output number beyond [-1, 1] is clamped by the
// conversion (to +-32767).  The step kernel tracks each converted pair and
// flags the solve if any value was clamped: with one node per thread by
// the largest |output number| (one three-way max per pair), with several by
// a packed max and min of the converted pairs (fewer live registers there).
template <bool PACKED>
struct SatTrack;
template <>
struct SatTrack<false> {
  float m = 0.0f;
  __device__ __forceinline__ void add(float a, float b, mrtlb_short2) {
    m = __builtin_fmaxf(m, __builtin_fmaxf(fabsf(a), fabsf(b)));
  }
  __device__ __forceinline__ bool any() const { return m > 1.0f; }
};
template <>
struct SatTrack<true> {
  mrtlb_short2 hi = {-32768, -32768}, lo = {32767, 32767};
  __device__ __forceinline__ void add(float, float, mrtlb_short2 v) {
    hi = __builtin_elementwise_max(hi, v);
    lo = __builtin_elementwise_min(lo, v);
  }
  __device__ __forceinline__ bool any() const {
    return (hi[0] == 32767) | (hi[1] == 32767) | (lo[0] == -32767) | (lo[1] == -32767);
  }
};

template <int ST, class Real>
__device__ __forceinline__ Real load_pop(const void* buf, uint32_t i, const KParams<Real>& P, int j) {
  using T = typename StoreT<ST>::T;
  return decode<ST>(gload<T>(buf, i * (uint32_t)sizeof(T)), P, j);
}

template <int ST, class Real>
__device__ __forceinline__ void store_pop(void* buf, uint32_t i, Real v, const KParams<Real>& P, int j) {
  using T = typename StoreT<ST>::T;
  gstore<T>(buf, i * (uint32_t)sizeof(T), encode<ST>(v, P, j));
}

// ---------------------------------------------------------------------------
// moments of a node
// ---------------------------------------------------------------------------

template <class Real>
struct Moments {
  Real R0;
  Real m1[3], m2n[3], m2o[3], m3m[3][3], m3p[3], mxyz;
};

// Component Hermite moments from the monomial sums of the populations in
// lattice units: R0 = sum f, R1_a = sum e_a f, R2n_a = sum e_a^2 f,
// R2o_ab = sum e_a e_b f, R3p_a = sum e_a^3 f, R3m_ab = sum e_a e_b^2 f,
// Rxyz = sum e_x e_y e_z f (PURE3 = false: no pure third-order rows).
template <int D, bool STANDARD, class Real>
__device__ __forceinline__ void finish_moments(const KParams<Real>& P, Real R0, const Real (&R1)[3],
                                               const Real (&R2n)[3], const Real (&R2o)[3], const Real (&R3p)[3],
                                               const Real (&R3m)[3][3], Real Rxyz, Moments<Real>& M) {
  M.R0 = R0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    M.m1[a] = P.c1[a] * R1[a];
    M.m2n[a] = P.c2[a] * R2n[a] - P.cs2 * R0;
  }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a + 1; b < D; ++b) M.m2o[off_index(a, b)] = P.cab[off_index(a, b)] * R2o[off_index(a, b)];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    Real pure = P.c3[a] * R3p[a] - 3 * P.cs2 * M.m1[a];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      if (b == a) continue;
      M.m3m[a][b] = P.cabb[a][b] * R3m[a][b] - P.cs2 * M.m1[a];
      pure -= P.corr[a][b] * M.m3m[a][b];
    }
    M.m3p[a] = STANDARD ? Real(0) : pure;
  }
  if constexpr (D == 3) M.mxyz = P.cxyz * Rxyz;
}

// Hermite moments (component rows, physical units) of x[0..B-1].  SCALED:
// x holds read numbers, population j is x_j * wsc[j] (one scale per pair).
// The monomial sums run over rays: the pairs of a ray have velocities
// sign * k * b for one direction b, so a degree-n monomial of a pair is
// (sign k)^n times that of b, and each ray needs the four partial sums
//   S0 = sum s, S2 = sum k^2 s, D1 = sum sign k d, D3 = sum sign k^3 d
// (s = f_p + f_q, d = f_p - f_q) before its monomials are added once.
// Accumulators start at -0.0, the additive identity the compiler folds.
template <class L, bool SCALED, class Real>
__device__ __forceinline__ void forward(const Real (&x)[L::B], const KParams<Real>& P, Moments<Real>& M) {
  constexpr int D = L::D;
  const Real z = Real(-0.0);
  Real R0 = SCALED ? x[0] * P.wsc[0] : x[0];
  Real R1[3] = {z, z, z}, R2n[3] = {z, z, z}, R2o[3] = {z, z, z}, R3p[3] = {z, z, z};
  Real R3m[3][3] = {{z, z, z}, {z, z, z}, {z, z, z}};
  Real Rxyz = z;
  static_for<0, n_pairs<L>()>([&](auto ll) {
    constexpr int lead = decltype(ll)::value;
    if constexpr (ray_leader<L>(lead) == lead) {
      Real S0 = z, S2 = z, D1 = z, D3 = z;
      static_for<lead, n_pairs<L>()>([&](auto kk) {
        constexpr int pp = decltype(kk)::value;
        if constexpr (ray_leader<L>(pp) == lead) {
          constexpr int p = pair_first<L>(pp);
          constexpr int q = opposite<L>(p);
          constexpr int k = ray_scale<L>(pp);
          constexpr int sk = ray_sign<L>(pp) * k;
          Real s = x[p] + x[q];
          Real d = x[p] - x[q];
          if constexpr (SCALED) {
            s *= P.wsc[p];
            d *= P.wsc[p];
          }
          S0 += s;
          S2 += Real(k * k) * s;
          D1 += Real(sk) * d;
          if constexpr (!is_standard<L>()) D3 += Real(sk * k * k) * d;
        }
      });
      R0 += S0;
      static_for<0, D>([&](auto aa) {
        constexpr int a = decltype(aa)::value;
        constexpr int ba = ray_dir<L>(lead, a);
        if constexpr (ba != 0) {
          // single layer (k = 1 on every ray): D3 = D1, and no pure rows
          const Real Dodd = is_standard<L>() ? D1 : D3;
          R1[a] += Real(ba) * D1;
          R2n[a] += Real(ba * ba) * S2;
          if constexpr (!is_standard<L>()) R3p[a] += Real(ba * ba * ba) * D3;
          static_for<0, D>([&](auto bb) {
            constexpr int b = decltype(bb)::value;
            constexpr int bv = ray_dir<L>(lead, b);
            if constexpr (b != a && bv != 0) R3m[a][b] += Real(ba * bv * bv) * Dodd;
            if constexpr (b > a && bv != 0) R2o[off_index(a, b)] += Real(ba * bv) * S2;
          });
        }
      });
      if constexpr (D == 3) {
        constexpr int bxyz = ray_dir<L>(lead, 0) * ray_dir<L>(lead, 1) * ray_dir<L>(lead, 2);
        if constexpr (bxyz != 0) Rxyz += Real(bxyz) * (is_standard<L>() ? D1 : D3);
      }
    }
  });
  finish_moments<D, is_standard<L>()>(P, R0, R1, R2n, R2o, R3p, R3m, Rxyz, M);
}

// Per-row coefficients delta_r = (target_r) / n_r turned into monomial
// coefficients in lattice units, then evaluated per velocity pair:
//   x_j <- kx * x_j + wo_j * sum_P beta_P e_j^P
// (wo = w for populations in physical units; see KParams for the 16-bit
// storages, whose output numbers it writes directly).  Per ray the even and
// odd parts are b0 + k^2 E2 and sign (k O1 + k^3 O3), with E2, O1, O3 the
// degree-2, -1 and -3 polynomials at the ray direction.
// Monomial coefficients (lattice units) of sum_r H_r delta_r for the
// targets delta_r = d*: f_j gains wo_j times
//   b0 + sum_a b1_a e_a + sum_a b2n_a e_a^2 + sum_{a<b} b2o_ab e_a e_b
//      + sum_a b3p_a e_a^3 + sum_{a!=b} b3m_ab e_a e_b^2 + bxyz e_x e_y e_z.
template <class Real>
struct BackCoeffs {
  Real b0, b1[3], b2n[3], b2o[3], b3m[3][3], b3p[3], bxyz;
};

template <int D, bool STANDARD, class Real>
__device__ __forceinline__ void back_coeffs(const KParams<Real>& P, Real d0, const Real* d1, const Real* d2n,
                                            const Real* d2o, const Real (*d3m)[3], const Real* d3p, Real dxyz,
                                            BackCoeffs<Real>& C) {
  C.b0 = d0;
#pragma unroll
  for (int a = 0; a < D; ++a) C.b0 -= P.cs2 * d2n[a];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    constexpr bool pure3 = !STANDARD;
    Real t = pure3 ? d1[a] + P.k3[a] * d3p[a] : d1[a];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      if (b == a) continue;
      t -= P.cs2 * d3m[a][b];
      C.b3m[a][b] = pure3 ? P.cabb[a][b] * (d3m[a][b] - P.corr[a][b] * d3p[a]) : P.cabb[a][b] * d3m[a][b];
    }
    C.b1[a] = P.c1[a] * t;
    C.b2n[a] = P.c2[a] * d2n[a];
    C.b3p[a] = pure3 ? P.c3[a] * d3p[a] : Real(0);
  }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = a + 1; b < D; ++b) C.b2o[off_index(a, b)] = P.cab[off_index(a, b)] * d2o[off_index(a, b)];
  C.bxyz = 0;
  if constexpr (D == 3) C.bxyz = P.cxyz * dxyz;
}

template <class L, class Real>
__device__ __forceinline__ void backward(Real (&x)[L::B], const KParams<Real>& P, Real kx, const Real* wo, Real d0,
                                         const Real* d1, const Real* d2n, const Real* d2o, const Real (*d3m)[3],
                                         const Real* d3p, Real dxyz) {
  constexpr int D = L::D;
  const Real z = Real(-0.0);
  BackCoeffs<Real> C;
  back_coeffs<D, is_standard<L>()>(P, d0, d1, d2n, d2o, d3m, d3p, dxyz, C);
  const Real b0 = C.b0, bxyz = C.bxyz;
  const auto& b1 = C.b1;
  const auto& b2n = C.b2n;
  const auto& b2o = C.b2o;
  const auto& b3m = C.b3m;
  const auto& b3p = C.b3p;
  x[0] = kx * x[0] + wo[0] * b0;
  static_for<0, n_pairs<L>()>([&](auto ll) {
    constexpr int lead = decltype(ll)::value;
    if constexpr (ray_leader<L>(lead) == lead) {
      Real E2 = z, O1 = z, O3 = z;
      static_for<0, D>([&](auto aa) {
        constexpr int a = decltype(aa)::value;
        constexpr int ba = ray_dir<L>(lead, a);
        if constexpr (ba != 0) {
          E2 += Real(ba * ba) * b2n[a];
          O1 += Real(ba) * b1[a];
          if constexpr (!is_standard<L>()) O3 += Real(ba * ba * ba) * b3p[a];
          static_for<0, D>([&](auto bb) {
            constexpr int b = decltype(bb)::value;
            constexpr int bv = ray_dir<L>(lead, b);
            if constexpr (b != a && bv != 0) O3 += Real(ba * bv * bv) * b3m[a][b];
            if constexpr (b > a && bv != 0) E2 += Real(ba * bv) * b2o[off_index(a, b)];
          });
        }
      });
      if constexpr (D == 3) {
        constexpr int b3 = ray_dir<L>(lead, 0) * ray_dir<L>(lead, 1) * ray_dir<L>(lead, 2);
        if constexpr (b3 != 0) O3 += Real(b3) * bxyz;
      }
      static_for<lead, n_pairs<L>()>([&](auto kk) {
        constexpr int pp = decltype(kk)::value;
        if constexpr (ray_leader<L>(pp) == lead) {
          constexpr int p = pair_first<L>(pp);
          constexpr int q = opposite<L>(p);
          constexpr int k = ray_scale<L>(pp);
          constexpr int sk = ray_sign<L>(pp) * k;
          const Real even = b0 + Real(k * k) * E2;
          const Real odd = Real(sk) * O1 + Real(sk * k * k) * O3;
          const Real wp = wo[p];
          x[p] = kx * x[p] + wp * (even + odd);
          x[q] = kx * x[q] + wp * (even - odd);
        }
      });
    }
  });
}

// Equilibrium Hermite moments (orders 1..3) from the conserved variables.
template <class L, class Real, int MODEL>
struct Equilibrium {
  Real e1[3], e2n[3], e2o[3], e3m[3][3], e3p[3], exyz;

  // NSE: j = rho_m u (momentum incl. the half force), u = j / rho_m.
  // NCDE: phi, u = advection velocity.
  __device__ __forceinline__ void build(const KParams<Real>& P, Real rho_or_phi, const Real* j, const Real* u) {
    constexpr int D = L::D;
    if constexpr (MODEL == kCde) {
      // diffusion-type equilibrium w_j phi: no Hermite moment above order 0
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        e1[a] = 0; e2n[a] = 0; e2o[a] = 0; e3p[a] = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) e3m[a][b] = 0;
      }
      exyz = 0;
      (void)P; (void)rho_or_phi; (void)j; (void)u;
    } else if constexpr (MODEL == kNcde) {
      const Real phi = rho_or_phi;
      const Real Phi = P.phi_coef * (phi + P.D2 * phi * phi * phi * Real(1.0 / 3.0));
#pragma unroll
      for (int a = 0; a < D; ++a) {
        e1[a] = phi * u[a];
        e2n[a] = P.cs2 * (Phi - phi) + e1[a] * u[a];
        e3p[a] = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) e3m[a][b] = 0;
      }
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a + 1; b < D; ++b) e2o[off_index(a, b)] = e1[a] * u[b];
      exyz = 0;
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        e1[a] = j[a];
        e2n[a] = j[a] * u[a];
      }
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a + 1; b < D; ++b) e2o[off_index(a, b)] = j[a] * u[b];
      // M30 = rho uuu (m30 = 1) or 0: a multiplier keeps this branch-free
      const Real g30 = P.m30 ? Real(1) : Real(0);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        Real pure = e2n[a] * u[a];
#pragma unroll
        for (int b = 0; b < D; ++b) {
          if (b == a) continue;
          e3m[a][b] = e2n[b] * u[a];  // rho u_a u_b^2
          pure -= P.corr[a][b] * e3m[a][b];
        }
        e3p[a] = is_standard<L>() ? Real(0) : g30 * pure;
#pragma unroll
        for (int b = 0; b < D; ++b) e3m[a][b] *= g30;
      }
      exyz = 0;
      if constexpr (D == 3) exyz = g30 * (j[0] * u[1] * u[2]);
    }
  }
};

// ---------------------------------------------------------------------------
// the fused collide-and-stream step
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t xcd_remap(uint32_t lin, uint32_t total) {
  // Workgroups are dealt to the XCDs round-robin; give every XCD a
  // contiguous range of tiles so that neighbouring tiles (which share
  // partially-read cache lines and halo rows) meet in the same L2.
  const uint32_t q = total / kNumXcd;
  if (lin >= q * kNumXcd) return lin;
  return (lin % kNumXcd) * q + lin / kNumXcd;
}

template <class Real>
__device__ __forceinline__ int find_job(const Job<Real>* jobs, int njobs, uint32_t lin) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block_begin <= lin) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Mapping of a step workgroup: the node slots of a solve are its rows laid
// end to end at the padded pitch nxp (a multiple of 32 nodes), cut into
// runs of kBlock * VEC slots; thread t of workgroup w owns the VEC
// consecutive slots starting at (w * kBlock + t) * VEC.  Every wavefront
// therefore starts on a 32-node boundary of a row (its accesses cover whole
// cache lines whatever nx is); slots past nx in a row are idle.
template <int VEC, class Real>
__device__ __forceinline__ bool tile_node(const Job<Real>& J, uint32_t local, int& ix0, int& iy, int& iz) {
  const uint32_t n0 = (local * (uint32_t)kBlock + threadIdx.x) * (uint32_t)VEC;
  const uint32_t nxp = (uint32_t)J.P.nxp, ny = (uint32_t)J.P.ny;
  const uint32_t r = n0 / nxp;
  ix0 = (int)(n0 - r * nxp);
  iy = (int)(r % ny);
  iz = (int)(r / ny);
  return ix0 < J.P.nx && r < ny * (uint32_t)J.P.nz;
}

// Relaxation targets of one node: f* = kx f + W sum_r H_r delta_r / n_r
// with the delta_r (scaled by 1/n_r) below.
template <class Real>
struct Targets {
  Real kx, d0, d1[3], d2n[3], d2o[3], d3m[3][3], d3p[3], dxyz;
};

// a2 and a4-a6 of one node in moment space: conserved variables, sources,
// equilibrium, relaxation.  M holds the node's Hermite moments on entry.
template <class L, int ST, int MODEL, bool FORCE>
__device__ __forceinline__ void relax_node(Moments<typename StoreT<ST>::Real>& M,
                                           const Job<typename StoreT<ST>::Real>& J, const RowGeom<L>& g, int ix,
                                           Targets<typename StoreT<ST>::Real>& T) {
  using Real = typename StoreT<ST>::Real;
  constexpr int D = L::D;
  const KParams<Real>& P = J.P;
  const uint32_t self = g.node(ix);
  const uint32_t N = P.N;
  // a8 drift correction (zero except on the step after an FP64 check): the
  // conserved moments enter the collision shifted by dm0, dm1, and the
  // targets below add (1 - s_h) dm to rows 0 and 1, whose (1 - s_h) f term
  // acts on the unshifted populations, so the step moves each node's totals
  // by exactly dm0 and dm1
  M.R0 += P.dm0;
#pragma unroll
  for (int a = 0; a < D; ++a) M.m1[a] += P.dm1[a];

  // a2: conserved variables, a5: sources
  Real F[3] = {0, 0, 0}, src1[3] = {0, 0, 0}, x1[3] = {0, 0, 0}, T2n[3] = {0, 0, 0}, T2o[3] = {0, 0, 0};
  Real h1[3] = {0, 0, 0};   // NSE three-level: hf (F(t) - F(t - dt)) after a force change
  Real u[3] = {0, 0, 0}, jm[3] = {0, 0, 0};
  const char* fbase = static_cast<const char*>(static_cast<const void*>(J.force));
  // NSE mass source at this node (forced kernels): the field or the uniform value
  Real Sm = 0;
  Real dS = 0;   // three-level scheme after a source change: hf (S(t) - S(t - dt))
  if constexpr (FORCE && MODEL != kNcde && MODEL != kCde) {
    Sm = P.msrc;
    if (P.sfield) Sm = gload<Real>(fbase + (size_t)D * N * sizeof(Real), self * (uint32_t)sizeof(Real));
  }
  // NCDE: phi from the sum and the source correction (eq. 2-4-1); NSE: rho
  // with the mass-source correction (eqs. 2-4-0, 2-4-2)
  const Real R = MODEL == kNcde ? (M.R0 + P.sqh) * P.sci : (FORCE ? M.R0 + P.rho_ref + P.cS * Sm : M.R0 + P.rho_ref);
  Real src0 = 0;   // source increment of the zeroth moment (NCDE source, NSE mass source)
  Real sg = 0;   // CDE: S_G = -u . grad(phi), grad(phi) = -s1 sum_j c_j f_j / cs^2
  if constexpr (MODEL == kCde) {
    const char* vel = static_cast<const char*>(static_cast<const void*>(J.force));
    Real dot = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
      dot += gload<Real>(vel + (size_t)a * N * sizeof(Real), self * (uint32_t)sizeof(Real)) * M.m1[a];
    sg = P.s1 * dot / P.cs2;
  } else if constexpr (MODEL == kNcde) {
    const Real phi_prev = gload<Real>(J.phi_prev, self * (uint32_t)sizeof(Real));
    Real adv = 0, grad[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
      u[a] = P.adv[a];
      grad[a] = (gload<Real>(J.phi_prev, g.shifted(ix, a, 1) * (uint32_t)sizeof(Real)) -
                 gload<Real>(J.phi_prev, g.shifted(ix, a, -1) * (uint32_t)sizeof(Real))) /
                (2 * P.c1[a]);
      adv += u[a] * grad[a];
    }
    const Real dphi = R - phi_prev;
    const Real scal = dphi + adv;
    src0 = P.sa * (P.sq + P.sk * R) + P.sp * (P.sq + P.sk * phi_prev);
    // M1G = (1 - s1/2) u scal - s1 X with X = A1 d_t(B_bar) + A2 div(D_bar)
    // of the general NCDE (gbt = gdd = 0: the plain NCDE)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      src1[a] = u[a] * scal;
      x1[a] = P.gbt[a] * dphi + P.gdd[a] * grad[a];
    }
    gstore<Real>(J.phi_out, self * (uint32_t)sizeof(Real), R);
  } else {
    if constexpr (FORCE) {
#pragma unroll
      for (int a = 0; a < D; ++a)
        F[a] = gload<Real>(fbase + (size_t)a * N * sizeof(Real), self * (uint32_t)sizeof(Real));
    }
    const Real rho_m = P.inc ? P.rho0 : R;
    const Real inv = Real(1) / rho_m;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      jm[a] = FORCE ? M.m1[a] + P.fh * F[a] : M.m1[a];
      u[a] = jm[a] * inv;
      src1[a] = F[a];
    }
    if constexpr (FORCE) {
      // uF + Fu, and for a mass source (cs^2 I - uu) S of M2G together with
      // the -cs^2 S I Hermite part of the source distribution (M0F = S): -uu S
#pragma unroll
      for (int a = 0; a < D; ++a) T2n[a] = 2 * u[a] * F[a] - Sm * u[a] * u[a];
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a + 1; b < D; ++b) T2o[off_index(a, b)] = u[a] * F[b] + u[b] * F[a] - Sm * u[a] * u[b];
      src0 = Sm;
      if (J.fprev) {
        // three-level scheme, the step after a change: hf (F(t) - F(t - dt))
        const char* pbase = static_cast<const char*>(static_cast<const void*>(J.fprev));
#pragma unroll
        for (int a = 0; a < D; ++a)
          h1[a] = P.hf * (F[a] - gload<Real>(pbase + (size_t)a * N * sizeof(Real), self * (uint32_t)sizeof(Real)));
        // the source's difference term: raw M0 only, so Hermite rows 0 and
        // (with -cs^2) the normal second-order ones
        if (P.sfield) {
          dS = P.hf * (Sm - gload<Real>(pbase + (size_t)D * N * sizeof(Real), self * (uint32_t)sizeof(Real)));
          src0 += dS;
        }
      }
    }
    if constexpr (MODEL == kNseGrad) {
      // gradient form of M2G_bar from the previous step's fields: the
      // backward difference in time and central differences in space
      const Real rp = gload<Real>(J.phi_prev, self * (uint32_t)sizeof(Real));
      if (P.inc) {
        // eq. M2G with p = cs^2 rho_bar, rho = rho0: T gains
        // u F_bar + F_bar u - uu S_bar minus its closed form,
        // F_bar - F = -cs^2 grad(rho_bar), S_bar - S = -d_t rho_bar
        const Real dtr = R - rp;
        Real gr[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < D; ++a)
          gr[a] = (gload<Real>(J.phi_prev, g.shifted(ix, a, 1) * (uint32_t)sizeof(Real)) -
                   gload<Real>(J.phi_prev, g.shifted(ix, a, -1) * (uint32_t)sizeof(Real))) /
                  (2 * P.c1[a]);
#pragma unroll
        for (int a = 0; a < D; ++a) T2n[a] += u[a] * (u[a] * dtr - 2 * P.cs2 * gr[a]);
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = a + 1; b < D; ++b)
            T2o[off_index(a, b)] += u[a] * u[b] * dtr - P.cs2 * (u[a] * gr[b] + u[b] * gr[a]);
      } else {
        // eq. M2G-1: (d_t p + div(p u)) I in place of cs^2 S I, p = cs^2 rho
        const char* jp = static_cast<const char*>(static_cast<const void*>(J.phi_prev));
        Real div = R - rp;
#pragma unroll
        for (int a = 0; a < D; ++a)
          div += (gload<Real>(jp + (size_t)(1 + a) * N * sizeof(Real), g.shifted(ix, a, 1) * (uint32_t)sizeof(Real)) -
                  gload<Real>(jp + (size_t)(1 + a) * N * sizeof(Real), g.shifted(ix, a, -1) * (uint32_t)sizeof(Real))) /
                 (2 * P.c1[a]);
        const Real extra = P.cs2 * (div - Sm);
#pragma unroll
        for (int a = 0; a < D; ++a) T2n[a] += extra;
        char* jo = static_cast<char*>(static_cast<void*>(J.phi_out));
#pragma unroll
        for (int a = 0; a < D; ++a) gstore<Real>(jo + (size_t)(1 + a) * N * sizeof(Real), self * (uint32_t)sizeof(Real), jm[a]);
      }
      gstore<Real>(J.phi_out, self * (uint32_t)sizeof(Real), R);
    }
  }

  // a4: equilibrium moments
  Equilibrium<L, Real, MODEL> E;
  E.build(P, R, jm, u);

  // a6: relaxation; targets t_r = m*_r - (1 - s_h) m_r, scaled by 1/n_r
  const Real kx = Real(1) - P.sh;
  Real d1[3], d2n[3], d2o[3], d3m[3][3], d3p[3], dxyz = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    Real ms = M.m1[a] - P.s1 * (M.m1[a] - E.e1[a]);
    if constexpr (FORCE || MODEL == kNcde) ms += P.g1 * src1[a] + h1[a];
    if constexpr (MODEL == kNcde) ms -= P.s1 * x1[a];
    d1[a] = (ms - kx * (M.m1[a] - P.dm1[a])) * P.in1[a];
  }
  {
    Real neq[3], tn = 0, tT = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      neq[a] = M.m2n[a] - E.e2n[a];
      tn += neq[a];
      tT += T2n[a];
    }
    tn *= Real(1.0 / D);
    tT *= Real(1.0 / D);
    const Real kb = Real(1) - P.sb, ks = Real(1) - P.ss;
    const Real gb = Real(1) - Real(0.5) * P.sb, gs = Real(1) - Real(0.5) * P.ss;
    if constexpr (is_standard<L>()) {
      // k = 1: the full normal block, m* = m_eq + (I - S2) neq + (I - S2/2) T
#pragma unroll
      for (int a = 0; a < D; ++a) {
        Real ms = E.e2n[a];
#pragma unroll
        for (int b = 0; b < D; ++b) {
          ms += P.k2[a][b] * neq[b];
          if constexpr (FORCE || MODEL == kNseGrad) ms += P.g2[a][b] * T2n[b];
        }
        if constexpr (FORCE) ms += P.kx2[a] * Sm - P.cs2 * dS;
        d2n[a] = (ms - kx * M.m2n[a]) * P.in2n[a];
      }
    } else {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        Real ms = E.e2n[a] + kb * tn + ks * (neq[a] - tn) + gb * tT + gs * (T2n[a] - tT);
        if constexpr (FORCE) ms += P.kx2[a] * Sm - P.cs2 * dS;
        d2n[a] = (ms - kx * M.m2n[a]) * P.in2n[a];
      }
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = a + 1; b < D; ++b) {
        const int o = off_index(a, b);
        const Real ms = E.e2o[o] + ks * (M.m2o[o] - E.e2o[o]) + gs * T2o[o];
        d2o[o] = (ms - kx * M.m2o[o]) * P.in2o[o];
      }
  }
  {
    const Real k3 = Real(1) - P.s3;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      d3p[a] = is_standard<L>() ? Real(0) : (E.e3p[a] + k3 * (M.m3p[a] - E.e3p[a]) - kx * M.m3p[a]) * P.in3p[a];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        if (b == a) continue;
        d3m[a][b] = (E.e3m[a][b] + k3 * (M.m3m[a][b] - E.e3m[a][b]) - kx * M.m3m[a][b]) * P.in3m[a][b];
      }
    }
    if constexpr (D == 3) dxyz = (E.exyz + k3 * (M.mxyz - E.exyz) - kx * M.mxyz) * P.inxyz;
  }
  // order 0 is conserved, m*_0 = m_0, except for the CDE source:
  // m*_0 = m_0 + M0G + s0 S_G / 2 = m_0 + S_G (M0G = (1 - s0/2) S_G)
  const Real d0 = (P.sh * M.R0 + kx * P.dm0 + sg + src0) * P.in0;
  T.kx = kx;
  T.d0 = d0;
  T.dxyz = dxyz;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    T.d1[a] = d1[a];
    T.d2n[a] = d2n[a];
    T.d3p[a] = d3p[a];
#pragma unroll
    for (int b = 0; b < D; ++b)
      if (b != a) T.d3m[a][b] = d3m[a][b];
  }
#pragma unroll
  for (int o = 0; o < D * (D - 1) / 2; ++o) T.d2o[o] = d2o[o];
}

// One node of the method after the gather: a2-a7 in registers.
// x[] holds the pre-collision populations on entry, post-collision on exit.
template <class L, int ST, int MODEL, bool FORCE>
__device__ __forceinline__ void collide_node(typename StoreT<ST>::Real (&x)[L::B],
                                             const Job<typename StoreT<ST>::Real>& J, const RowGeom<L>& g, int ix) {
  using Real = typename StoreT<ST>::Real;
  const KParams<Real>& P = J.P;
  // a3: forward Hermite moments
  Moments<Real> M;
  forward<L, scaled_storage<ST>()>(x, P, M);
  Targets<Real> T;
  relax_node<L, ST, MODEL, FORCE>(M, J, g, ix, T);
  // a7: back to populations (output numbers of the storage)
  backward<L>(x, P, T.kx * P.kin, P.wo, T.d0, T.d1, T.d2n, T.d2o, T.d3m, T.d3p, T.dxyz);
}

// a1 of VEC consecutive nodes of a row: f_bar_j(x, t) read from the row of
// x - e_j.  The rest population (e = 0) is read at the own node; population
// j >= 1 at a wave-uniform base (soffset) plus a lane offset that depends on
// the source row only (RowGeom); at the periodic x-edges the wrapped
// elements are loaded one by one with one lane offset per distinct e_x.
template <class L, int ST, int VEC, bool UNIROW>
__device__ __forceinline__ void gather(const Job<typename StoreT<ST>::Real>& J, const RowGeom<L>& g, int ix0,
                                       typename StoreT<ST>::T (&raw)[L::B][VEC]) {
  using T = typename StoreT<ST>::T;
  constexpr int B = L::B;
  constexpr int M = L::MAXE;
  static_assert(L::EX[0] == 0 && L::EY[0] == 0, "population 0 is the rest velocity");
  const auto& P = J.P;
  const auto rin = make_rsrc(J.fin, P.pop_bytes);
  // one node per lane: a wave-uniform choice, so no wave runs both paths
  const bool inside = ix0 >= M && ix0 + VEC - 1 + M < P.nx;
  const bool interior = VEC == 1 ? __all(inside) != 0 : inside;
  // With UNIROW the wave lies in one grid row (g built from wave-uniform
  // y, z): every source row offset is wave-uniform and rides in soffset
  // with the population's own uniform part, and the lane part is x alone.
  auto split = [&](uint32_t uni, uint32_t row, uint32_t x, uint32_t& u, uint32_t& l) {
    if constexpr (UNIROW) {
      u = uni + row;
      l = x;
    } else {
      u = uni;
      l = row + x;
    }
  };
  if (interior) {
    // whole VEC-runs inside the row: the lane part depends on the row only
    const uint32_t lx = (uint32_t)(ix0 + M);
    uint32_t u, l;
    split(0u, g.lown(), (uint32_t)ix0, u, l);
    load_vec<ST, VEC>(rin, u, l, raw[0]);
    static_for<1, B>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      uint32_t uj, lj;
      split(g.template uni_src<j>(), g.template lrow<j>(), lx, uj, lj);
      load_vec<ST, VEC>(rin, uj, lj, raw[j]);
    });
  } else {
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      uint32_t lx[2 * M + 1];
#pragma unroll
      for (int e = -M; e <= M; ++e) lx[e + M] = (uint32_t)(wrap(ix0 + k - e, P.nx) + e + M);
      T one[1];
      uint32_t u, l;
      split(0u, g.lown(), (uint32_t)(ix0 + k), u, l);
      load_vec<ST, 1>(rin, u, l, one);
      raw[0][k] = one[0];
      static_for<1, B>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        uint32_t uj, lj;
        split(g.template uni_src<j>(), g.template lrow<j>(), lx[L::EX[j] + M], uj, lj);
        load_vec<ST, 1>(rin, uj, lj, one);
        raw[j][k] = one[0];
      });
    }
  }
}

// a1 for the node run (ix0 .. ix0 + VEC - 1) of row (iy, iz).  When the row
// pitch is a multiple of the slots of a wave, no wave crosses a grid row:
// the source rows are wave-uniform and their offsets are computed once per
// wave on the scalar unit.
template <class L, int ST, int VEC>
__device__ __forceinline__ void gather_run(const Job<typename StoreT<ST>::Real>& J, const RowGeom<L>& g, int ix0,
                                           int iy, int iz, typename StoreT<ST>::T (&raw)[L::B][VEC]) {
  const auto& P = J.P;
  if (P.nxp % (64 * VEC) == 0) {
    RowGeom<L> gw;
    gw.init(__builtin_amdgcn_readfirstlane(iy), __builtin_amdgcn_readfirstlane(iz), P.nx, P.nxp, P.ny, P.nz);
    gather<L, ST, VEC, true>(J, gw, ix0, raw);
  } else {
    gather<L, ST, VEC, false>(J, g, ix0, raw);
  }
}

// a8: VEC-wide aligned stores of the run at the own nodes
template <class L, int ST, int VEC>
__device__ __forceinline__ void store_run(const Job<typename StoreT<ST>::Real>& J, const RowGeom<L>& g, int ix0,
                                          const typename StoreT<ST>::T (&raw)[L::B][VEC]) {
  const auto rout = make_rsrc(J.fout, J.P.pop_bytes);
  const uint32_t lo = g.lown() + (uint32_t)ix0;
  static_for<0, L::B>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    store_vec<ST, VEC>(rout, (uint32_t)j * (uint32_t)J.P.nxp, lo, raw[j]);
  });
}

// ---------------------------------------------------------------------------
// the fused collide-and-stream step: every thread owns VEC consecutive nodes
// along x.  a1: each population is gathered with one VEC-wide load from the
// row of x - e_j (element-aligned: the pull shift); at the periodic x-edges
// the wrapped elements are loaded one by one.  a8: VEC-wide aligned stores at
// the own nodes.
// ---------------------------------------------------------------------------

template <class L, int ST, int MODEL, bool FORCE, int VEC>
__global__ __launch_bounds__(kBlock) void k_step(const Job<typename StoreT<ST>::Real>* __restrict__ jobs, int njobs,
                                                uint32_t total_blocks) {
  using Real = typename StoreT<ST>::Real;
  using T = typename StoreT<ST>::T;
  constexpr int B = L::B;
  const uint32_t lin = xcd_remap(blockIdx.x, total_blocks);
  const int jb = njobs > 1 ? find_job(jobs, njobs, lin) : 0;
  const Job<Real>& J = jobs[jb];
  const KParams<Real>& P = J.P;
  int ix0, iy, iz;
  if (!tile_node<VEC>(J, lin - J.block_begin, ix0, iy, iz)) return;
  RowGeom<L> g;
  g.init(iy, iz, P.nx, P.nxp, P.ny, P.nz);

  // a1: gather along -e_j
  T raw[B][VEC];
  gather_run<L, ST, VEC>(J, g, ix0, iy, iz, raw);

  // a2-a7 in registers: x holds the numbers the storage reads as, the
  // back-transform leaves the numbers it writes (equal for FP32/FP64).  The
  // int16 format converts two nodes per instruction: an even node's output
  // waits in keep[] for the odd one.
  Real keep[ST == kI16Dev && VEC > 1 ? B : 1];
  SatTrack<(VEC > 1)> sat;
  static_for<0, VEC>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    Real x[B];
    static_for<0, B>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      x[j] = units<ST>(raw[j][k]);
    });
    collide_node<L, ST, MODEL, FORCE>(x, J, g, ix0 + k);
    static_for<0, B>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      if constexpr (ST == kI16Dev && VEC == 1) {
        // one node: populations j - 1 and j share a conversion
        if constexpr (j % 2 == 1) {
          const mrtlb_short2 r = snorm16x2(x[j - 1], x[j]);
          sat.add(x[j - 1], x[j], r);
          raw[j - 1][0] = r[0];
          raw[j][0] = r[1];
        } else if constexpr (j == B - 1) {
          const mrtlb_short2 r = snorm16x2(x[j], 0.0f);
          sat.add(x[j], 0.0f, r);
          raw[j][0] = r[0];
        }
      } else if constexpr (ST == kI16Dev && k % 2 == 0) {
        keep[j] = x[j];
      } else if constexpr (ST == kI16Dev) {
        const mrtlb_short2 r = snorm16x2(keep[j], x[j]);
        sat.add(keep[j], x[j], r);
        raw[j][k - 1] = r[0];
        raw[j][k] = r[1];
      } else {
        raw[j][k] = to_stored<ST>(x[j]);
      }
    });
  });

  // int16: a conversion clamped at +-1 gives +-32767; flag the solve
  if constexpr (ST == kI16Dev) {
    if (sat.any()) *J.sat = 1;
  }

  // a8: store at the own nodes
  store_run<L, ST, VEC>(J, g, ix0, raw);
}

// Streaming alone (eq. 2-2 with no collision): every stored number moves from
// x - e_j to x unchanged.  The step kernel's tiles, gather, tile order and
// store policy with nothing between them, so its rate is the ceiling of the
// step kernel's memory access pattern on the same grid.  One job.
template <class L, int ST, int VEC>
__global__ __launch_bounds__(kBlock) void k_stream(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                  uint32_t total_blocks) {
  const uint32_t lin = xcd_remap(blockIdx.x, total_blocks);
  const auto& J = jobs[0];
  const auto& P = J.P;
  int ix0, iy, iz;
  if (!tile_node<VEC>(J, lin, ix0, iy, iz)) return;
  RowGeom<L> g;
  g.init(iy, iz, P.nx, P.nxp, P.ny, P.nz);
  typename StoreT<ST>::T raw[L::B][VEC];
  gather_run<L, ST, VEC>(J, g, ix0, iy, iz, raw);
  store_run<L, ST, VEC>(J, g, ix0, raw);
}

// ---------------------------------------------------------------------------
// initialisation, read-out and restore: one thread per node (1D over nodes),
// computed in FP64 regardless of the storage.
// ---------------------------------------------------------------------------

template <class L>
__device__ __forceinline__ bool node_of_thread(const KParams<double>& P, int& ix, int& iy, int& iz) {
  const uint32_t n = blockIdx.x * (uint32_t)kBlock + threadIdx.x;
  if (n >= P.N) return false;
  const uint32_t nx = (uint32_t)P.nx, ny = (uint32_t)P.ny;
  ix = (int)(n % nx);
  iy = (int)((n / nx) % ny);
  iz = (int)(n / (nx * ny));
  return true;
}

// f_bar(x,0) = f_eq - F/2, written at x - e_j (inverse of the pull gather).
template <class L, int ST, int MODEL>
__global__ __launch_bounds__(kBlock) void k_init(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                const KParams<double>* __restrict__ PD, const double* __restrict__ rho,
                                                const double* __restrict__ uin, const double* __restrict__ fin,
                                                uint32_t total_blocks) {
  using Real = typename StoreT<ST>::Real;
  constexpr int B = L::B, D = L::D;
  const Job<Real>& J = jobs[0];
  const KParams<double>& P = *PD;
  int ix, iy, iz;
  if (!node_of_thread<L>(P, ix, iy, iz)) return;
  RowGeom<L> g;
  g.init(iy, iz, P.nx, P.nxp, P.ny, P.nz);
  const uint32_t self = g.node(ix);
  const uint32_t N = P.N;
  const double R = rho[self];
  double u[3] = {0, 0, 0}, jm[3] = {0, 0, 0}, F[3] = {0, 0, 0};
  double Sm = 0;    // NSE mass source at this node
  if constexpr (MODEL == kCde) {
    // equilibrium w_j phi; the velocity field is stored by the host
  } else if constexpr (MODEL == kNcde) {
    for (int a = 0; a < D; ++a) u[a] = P.adv[a];
    static_cast<Real*>(J.phi_out)[self] = (Real)R;
    const_cast<Real*>(J.phi_prev)[self] = (Real)R;
  } else {
    const double rho_m = P.inc ? P.rho0 : R;
    for (int a = 0; a < D; ++a) {
      u[a] = uin[(size_t)a * N + self];
      jm[a] = rho_m * u[a];
      if (fin) F[a] = fin[(size_t)a * N + self];
    }
    if (J.force) Sm = P.sfield ? (double)J.force[(size_t)D * N + self] : P.msrc;
    if constexpr (MODEL == kNseGrad) {
      // the history before t = 0 from the continuity equation:
      // rho^{-1} = rho^0 - S + div(rho_m u)^0 (central), (rho u)^{-1} = (rho u)^0,
      // in both slots
      double div = 0;
      for (int a = 0; a < D; ++a) {
        const uint32_t xp = g.shifted(ix, a, 1), xm = g.shifted(ix, a, -1);
        const double rp = P.inc ? P.rho0 : rho[xp], rm = P.inc ? P.rho0 : rho[xm];
        div += (rp * uin[(size_t)a * N + xp] - rm * uin[(size_t)a * N + xm]) / (2 * P.c1[a]);
      }
      Real* h0 = static_cast<Real*>(J.phi_out);
      Real* h1 = const_cast<Real*>(J.phi_prev);
      h0[self] = h1[self] = (Real)(R - Sm + div);
      if (!P.inc)
        for (int a = 0; a < D; ++a) h0[(size_t)(1 + a) * N + self] = h1[(size_t)(1 + a) * N + self] = (Real)jm[a];
    }
  }
  Equilibrium<L, double, MODEL> E;
  E.build(P, R, jm, u);
  double d1[3], d2n[3], d2o[3], d3m[3][3], d3p[3], dxyz = 0;
  for (int a = 0; a < D; ++a) {
    d1[a] = (E.e1[a] - P.fh * F[a]) * P.in1[a];
    d2n[a] = E.e2n[a] * P.in2n[a];
    d3p[a] = E.e3p[a] * P.in3p[a];
    for (int b = 0; b < D; ++b)
      if (b != a) d3m[a][b] = E.e3m[a][b] * P.in3m[a][b];
    for (int b = a + 1; b < D; ++b) d2o[off_index(a, b)] = E.e2o[off_index(a, b)] * P.in2o[off_index(a, b)];
  }
  if constexpr (D == 3) dxyz = E.exyz * P.inxyz;
  double x[B];
  for (int j = 0; j < B; ++j) x[j] = 0;
  // NCDE, full correction: f_bar = f_eq - w S(phi0) / 2
  // NSE: f_bar = f_eq minus the distribution of raw moments (cS S, fh F, 0)
  // (Hermite second order -cs^2 cS S); the F route: F/2 with M0F = S
  const double msh = P.cS * Sm;
  const double r0 = MODEL == kNcde ? R - P.sinit * (P.sq + P.sk * R) : R - msh;
  if constexpr (MODEL != kNcde && MODEL != kCde)
    for (int a = 0; a < D; ++a) d2n[a] += msh * P.cs2 * P.in2n[a];
  const double d0 = r0 * P.in0 - P.rho_ref;
  backward<L>(x, P, 0.0, P.w, d0, d1, d2n, d2o, d3m, d3p, dxyz);
  const KParams<Real>& PR = J.P;
  float smax = 0.0f;
  static_for<0, B>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    // buf_j(x - e_j) = f_bar_j(x): the source index of the pull gather
    smax = fmaxf(smax, sat_of<ST>((Real)x[j], PR, j));
    store_pop<ST>(J.fout, g.template src<j>(ix), (Real)x[j], PR, j);
  });
  raise_saturation<ST>(J, smax);
}

// read-out: gather f_bar(x, t) and compute moments (WHAT 0) or copy the
// populations (WHAT 1)
template <class L, int ST, int MODEL, int WHAT>
__global__ __launch_bounds__(kBlock) void k_gather(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                  const KParams<double>* __restrict__ PD, double* __restrict__ out0,
                                                  double* __restrict__ out1) {
  constexpr int B = L::B, D = L::D;
  const auto& J = jobs[0];
  const KParams<double>& P = *PD;
  int ix, iy, iz;
  if (!node_of_thread<L>(P, ix, iy, iz)) return;
  RowGeom<L> g;
  g.init(iy, iz, P.nx, P.nxp, P.ny, P.nz);
  const uint32_t self = g.node(ix);
  const uint32_t N = P.N;
  double x[B];
  static_for<0, B>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    x[j] = (double)load_pop<ST>(J.fin, g.template src<j>(ix), J.P, j);
  });
  if constexpr (WHAT == 1) {
    for (int j = 0; j < B; ++j) out0[(size_t)j * N + self] = x[j] + P.w[j] * P.rho_ref;
  } else {
    double R = 0, m1[3] = {0, 0, 0};
    static_for<0, B>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      R += x[j];
      static_for<0, D>([&](auto aa) {
        constexpr int a = decltype(aa)::value;
        if constexpr (evel<L>(j, a) != 0) m1[a] += double(evel<L>(j, a)) * x[j];
      });
    });
    R += P.rho_ref;
    if constexpr (MODEL == kCde) {
      // phi = sum_j f_j + S_G / 2; u is the stored velocity field
      double dot = 0;
      for (int a = 0; a < D; ++a) dot += (double)J.force[(size_t)a * N + self] * P.c1[a] * m1[a];
      out0[self] = R + 0.5 * P.s1 * dot / P.cs2;
      if (out1)
        for (int a = 0; a < D; ++a) out1[(size_t)a * N + self] = (double)J.force[(size_t)a * N + self];
      return;
    }
    if constexpr (MODEL != kNcde)
      if (J.force) R += P.cS * (P.sfield ? (double)J.force[(size_t)D * N + self] : P.msrc);
    out0[self] = MODEL == kNcde ? (R + P.sqh) * P.sci : R;
    if (out1) {
      if constexpr (MODEL == kNcde) {
        for (int a = 0; a < D; ++a) out1[(size_t)a * N + self] = P.adv[a];
      } else {
        const double rho_m = P.inc ? P.rho0 : R;
        for (int a = 0; a < D; ++a) {
          double jmom = P.c1[a] * m1[a];
          if (J.force) jmom += P.fh * (double)J.force[(size_t)a * N + self];
          out1[(size_t)a * N + self] = jmom / rho_m;
        }
      }
    }
  }
}

// Restore: buf_j(x - e_j) = f_bar_j(x) - w_j rho_ref.
template <class L, int ST>
__global__ __launch_bounds__(kBlock) void k_scatter(const Job<typename StoreT<ST>::Real>* __restrict__ jobs,
                                                   const KParams<double>* __restrict__ PD, const double* __restrict__ in) {
  using Real = typename StoreT<ST>::Real;
  constexpr int B = L::B;
  const Job<Real>& J = jobs[0];
  const KParams<double>& P = *PD;
  int ix, iy, iz;
  if (!node_of_thread<L>(P, ix, iy, iz)) return;
  RowGeom<L> g;
  g.init(iy, iz, P.nx, P.nxp, P.ny, P.nz);
  const uint32_t self = g.node(ix);
  const uint32_t N = P.N;
  float smax = 0.0f;
  static_for<0, B>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    const double v = in[(size_t)j * N + self] - P.w[j] * P.rho_ref;
    smax = fmaxf(smax, sat_of<ST>((Real)v, J.P, j));
    store_pop<ST>(J.fout, g.template src<j>(ix), (Real)v, J.P, j);
  });
  raise_saturation<ST>(J, smax);
}

// ---------------------------------------------------------------------------
// FP64 plane sums (conserved quantities): partial[plane][chunk] over chunks
// of kBlock * kChunkIters elements, wavefront shuffles then a fixed LDS tree.
// ---------------------------------------------------------------------------


template <int ST>
__global__ __launch_bounds__(kBlock) void k_plane_sums(const void* __restrict__ base, uint32_t N, int nplanes_pop,
                                                      const typename StoreT<ST>::Real* __restrict__ force, int nforce,
                                                      const KParams<typename StoreT<ST>::Real>* __restrict__ PR,
                                                      double* __restrict__ partial, uint32_t nchunks) {
  using Real = typename StoreT<ST>::Real;
  using T = typename StoreT<ST>::T;
  const uint32_t chunk = blockIdx.x;
  const int plane = blockIdx.y;
  const uint32_t begin = chunk * (uint32_t)(kBlock * kChunkIters);
  double acc = 0;
  for (int it = 0; it < kChunkIters; ++it) {
    const uint32_t i = begin + (uint32_t)it * kBlock + threadIdx.x;
    if (i < N) {
      if (plane < nplanes_pop) {
        const uint32_t nx = (uint32_t)PR->nx;
        const uint32_t e = ((i / nx) * (uint32_t)nplanes_pop + (uint32_t)plane) * (uint32_t)PR->nxp + i % nx;
        acc += (double)load_pop<ST>(base, e, *PR, plane);
      } else {
        acc += (double)force[(size_t)(plane - nplanes_pop) * N + i];
      }
    }
  }
  // wavefront reduction (64 lanes), fixed butterfly order
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ double red[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int k = 0; k < kBlock / 64; ++k) s += red[k];
    partial[(size_t)plane * nchunks + chunk] = s;
  }
}

// ---------------------------------------------------------------------------
// host launchers for one lattice
// ---------------------------------------------------------------------------

template <class F>
inline bool with_storage(int st, F&& f) {
  switch (st) {
    case kFP64: f(std::integral_constant<int, kFP64>{}); return true;
    case kFP32: f(std::integral_constant<int, kFP32>{}); return true;
    case kFP32Dev: f(std::integral_constant<int, kFP32Dev>{}); return true;
    case kFP16Dev: f(std::integral_constant<int, kFP16Dev>{}); return true;
    case kBF16Dev: f(std::integral_constant<int, kBF16Dev>{}); return true;
    case kI16Dev: f(std::integral_constant<int, kI16Dev>{}); return true;
    case kFP32DevF64: f(std::integral_constant<int, kFP32DevF64>{}); return true;
  }
  return false;
}

}  // namespace mrtlb
