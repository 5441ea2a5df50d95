// Device helpers shared by the gfx950 kernels.
//
// Amplitudes are interleaved complex (double2 for complex128, float2 for
// complex64).  Sweeps compute in the amplitude precision; every reduction
// (energy, norm, gradient) promotes products to FP64 and sums them in a fixed
// order: per lane, then across the 64 lanes of a wavefront, then across the
// wavefronts of a block in index order, then across blocks in index order,
// so these sums are bitwise reproducible for given inputs.  The lambda = H psi
// build adds into an FP64 accumulator tile in which every element is owned by
// one wavefront per segment of groups and updated in group order, so it is
// reproducible as well.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "q2sv_internal.h"

namespace q2sv {

// A real amplitude (SV_R64): the real part alone, 8 bytes.  Its imaginary
// part reads as a constant zero, so the complex arithmetic of every kernel
// instantiated on it folds to real arithmetic; code that would store an
// imaginary part stores nothing (cmake) or is written for it (is_real_amp).
struct R64 {
  double x;
  static constexpr double y = 0.0;
};

template <typename T> struct Real;
template <> struct Real<double2> { using type = double; };
template <> struct Real<float2> { using type = float; };
template <> struct Real<R64> { using type = double; };

template <typename T> inline constexpr bool is_real_amp = false;
template <> inline constexpr bool is_real_amp<R64> = true;

// Host dispatch on the amplitude type of a state (SV_C128, SV_C64, SV_R64):
// f receives a value of that type and launches with it.
template <typename F>
inline hipError_t by_dtype(int dtype, F&& f) {
  if (dtype == 0) f(double2{});
  else if (dtype == 1) f(float2{});
  else f(R64{});
  return hipGetLastError();
}

template <typename V>
__device__ __forceinline__ V cmake(typename Real<V>::type re, typename Real<V>::type im) {
  V v;
  v.x = re;
  if constexpr (!is_real_amp<V>) v.y = im;
  return v;
}

// v * i^e for e in 0..3
template <typename V>
__device__ __forceinline__ V mul_ipow(V v, unsigned e) {
  switch (e & 3u) {
    case 0: return v;
    case 1: return cmake<V>(-v.y, v.x);
    case 2: return cmake<V>(-v.x, -v.y);
    default: return cmake<V>(v.y, -v.x);
  }
}

__device__ __forceinline__ unsigned parity64(uint64_t v) { return __popcll(v) & 1u; }
__device__ __forceinline__ unsigned parity32(uint32_t v) { return __popc(v) & 1u; }

__device__ __forceinline__ uint64_t insert_zero(uint64_t t, unsigned pos) {
  const uint64_t low = t & ((uint64_t(1) << pos) - 1);
  return ((t >> pos) << (pos + 1)) | low;
}

// Insert zeros at ascending positions (final positions of the zero bits),
// packed one byte per position.
__device__ __forceinline__ uint64_t insert_zeros(uint64_t t, uint64_t pack, int n) {
  for (int j = 0; j < n; ++j) t = insert_zero(t, unsigned(pack >> (8 * j)) & 0xffu);
  return t;
}

__device__ __forceinline__ unsigned pack_at(uint64_t pack, int j) { return unsigned(pack >> (8 * j)) & 0xffu; }

__device__ __forceinline__ uint32_t insert_zero32(uint32_t t, unsigned pos) {
  const uint32_t low = t & ((1u << pos) - 1u);
  return ((t >> pos) << (pos + 1)) | low;
}

__device__ __forceinline__ uint32_t insert_zeros32(uint32_t t, uint64_t pack, int n) {
  for (int j = 0; j < n; ++j) t = insert_zero32(t, unsigned(pack >> (8 * j)) & 0xffu);
  return t;
}

// As above for frame-local positions (< 16) packed four bits each (up to 16).
__device__ __forceinline__ uint32_t insert_zeros32_p4(uint32_t t, uint64_t pack, int n) {
  for (int j = 0; j < n; ++j) t = insert_zero32(t, unsigned(pack >> (4 * j)) & 0xfu);
  return t;
}

// An empty use that needs v in an SGPR here: scalar loads feeding it all
// leave before this point (and are waited for once) instead of being sunk
// one by one into the branches that first use them.
__device__ __forceinline__ void sgpr_here(uint32_t v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void sgpr_here(uint64_t v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void sgpr_here(double v) { asm volatile("" ::"s"(v)); }

// ---------------------------------------------------------------------------
// deterministic FP64 reductions
// ---------------------------------------------------------------------------
// FP64 add into LDS that returns nothing (no wait on the old value).
__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------------------------------------------------------
// order-independent sums in fixed point
// ---------------------------------------------------------------------------
// For |x| < 2^51, t = x + 1.5 * 2^52 lies in [2^52, 2^53), where consecutive
// doubles are 1 apart: forming t rounds x to an integer q, and t's bit
// pattern minus that of 1.5 * 2^52 (whose low word is zero) is q in two's
// complement.  Integer adds are associative, so a sum of such q comes out
// the same in any order of arrival.
constexpr double kFxMagic = 6755399441055744.0;  // 1.5 * 2^52
constexpr int kFxNone = -4000;                   // exponent of a zero tile

__device__ __forceinline__ unsigned long long fx_bits(double t) {
  const uint32_t hi = uint32_t(__double2hiint(t)) - 0x43380000u;
  return (static_cast<unsigned long long>(hi) << 32) | uint32_t(__double2loint(t));
}

// Integer add into LDS that returns nothing; t = x * scale + kFxMagic.
__device__ __forceinline__ void lds_add_fx(unsigned long long* p, double t) {
  __hip_atomic_fetch_add(p, fx_bits(t), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// e with 2^(e-1) <= a < 2^e for a > 0; kFxNone for a = 0
__device__ __forceinline__ int fx_exp(double a) {
  return a > 0.0 ? __builtin_amdgcn_frexp_exp(a) : kFxNone;
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// One DPP data movement of a double (both halves); lanes the pattern does
// not feed, or rows row_mask leaves out, read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront (every lane active), returned to all
// lanes: inclusive scans within rows of 16 by row shifts, then the row totals
// carried by row broadcasts, so the total lands in lane 63.  Only VALU data
// movement (no LDS crossbar), and a fixed order of additions.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0x111, 0xf>(v);  // row_shr:1
  v += dpp_f64<0x112, 0xf>(v);  // row_shr:2
  v += dpp_f64<0x114, 0xf>(v);  // row_shr:4
  v += dpp_f64<0x118, 0xf>(v);  // row_shr:8
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sum over each row of 16 lanes, valid in the row's last lane (15, 31, 47,
// 63): the first four steps of wave_sum.
__device__ __forceinline__ double row_sum(double v) {
  v += dpp_f64<0x111, 0xf>(v);  // row_shr:1
  v += dpp_f64<0x112, 0xf>(v);  // row_shr:2
  v += dpp_f64<0x114, 0xf>(v);  // row_shr:4
  v += dpp_f64<0x118, 0xf>(v);  // row_shr:8
  return v;
}

// Sum over the block; result valid in thread 0.  `scratch` holds one double
// per wavefront.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < NW; ++w) s += scratch[w];
  }
  return s;
}

// ---------------------------------------------------------------------------
// frames: frame-local index l (B bits) -> global index base | deposit(l)
// ---------------------------------------------------------------------------
struct FrameLut {
  // deposit of frame-local bits [c, c + k1) and [c + k1, B) to global positions
  uint64_t lo[128];
  uint64_t hi[128];
  int c, k1, b;
};

// Deposit of the tile-block index into the complementary positions, walking
// the set bits of the mask: with a uniform index this stays on the scalar
// unit and touches no memory (a byte-table lookup would be a vector load,
// whose wait would also drain the tile loads and stores in flight).
__device__ __forceinline__ uint64_t frame_base(const FrameDesc& fr, uint64_t tb) {
  uint64_t base = 0;
  for (uint64_t m = fr.comp_mask; m; m &= m - 1, tb >>= 1)
    if (tb & 1ull) base |= m & (~m + 1ull);
  return base;
}

template <int NT>
__device__ void frame_lut_init(const FrameDesc& fr, FrameLut& lut) {
  const int c = fr.c, b = fr.b;
  const int rest = b - c;
  const int k1 = rest < 7 ? rest : 7;
  const int k2 = rest - k1;
  for (int i = threadIdx.x; i < (1 << k1); i += NT) {
    uint64_t g = 0;
    for (int j = 0; j < k1; ++j) g |= uint64_t((i >> j) & 1) << fr.q[c + j];
    lut.lo[i] = g;
  }
  for (int i = threadIdx.x; i < (1 << k2); i += NT) {
    uint64_t g = 0;
    for (int j = 0; j < k2; ++j) g |= uint64_t((i >> j) & 1) << fr.q[c + k1 + j];
    lut.hi[i] = g;
  }
  if (threadIdx.x == 0) {
    lut.c = c;
    lut.k1 = k1;
    lut.b = b;
  }
}

__device__ __forceinline__ uint64_t frame_deposit(const FrameLut& lut, uint32_t l) {
  const uint32_t cm = (1u << lut.c) - 1u;
  const uint32_t m1 = (1u << lut.k1) - 1u;
  return uint64_t(l & cm) | lut.lo[(l >> lut.c) & m1] | lut.hi[l >> (lut.c + lut.k1)];
}

// Register staging of PER amplitudes per thread, kept as separate real and
// imaginary scalar arrays so they stay in VGPRs.
template <typename T, int PER>
struct Stage {
  typename Real<T>::type re[PER];
  typename Real<T>::type im[PER];
};

// Issue the loads of one tile-block into registers (all loads in flight at
// once); thread t holds frame-local indices t, t + NT, ...
__device__ __forceinline__ uint32_t lds_swz(uint32_t l) { return lds_slot(l); }

// Bits of v deposited on the set bits of mask, ascending (uniform operands
// keep this on the scalar unit).
__device__ __forceinline__ uint32_t deposit_bits(uint32_t v, uint32_t mask) {
  uint32_t out = 0;
  for (uint32_t m = mask; m; m &= m - 1, v >>= 1)
    if (v & 1u) out |= m & (~m + 1u);
  return out;
}

// this wavefront's region bits: its index deposited into a segment's mask
__device__ __forceinline__ uint32_t region_bits_of(uint32_t wb_mask, uint32_t wave) {
  uint32_t wbits = 0;
  int j = 0;
  for (uint32_t m = wb_mask; m; m &= m - 1, ++j) wbits |= ((wave >> j) & 1u) << (__ffs(m) - 1);
  return wbits;
}

template <typename T, int PER, int NT>
__device__ __forceinline__ void tile_fetch(const T* __restrict__ src, const FrameLut& lut, uint64_t base,
                                           uint32_t nloc, Stage<T, PER>& reg) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const uint32_t l = threadIdx.x + uint32_t(i) * NT;
    if (l < nloc) {
      const T v = src[base | frame_deposit(lut, l)];
      reg.re[i] = v.x;
      reg.im[i] = v.y;
    }
  }
}

template <typename T, int PER, int NT>
__device__ __forceinline__ void tile_put(T* tile, uint32_t nloc, const Stage<T, PER>& reg) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const uint32_t l = threadIdx.x + uint32_t(i) * NT;
    if (l < nloc) tile[lds_swz(l)] = cmake<T>(reg.re[i], reg.im[i]);
  }
}

template <typename T, int PER, int NT>
__device__ __forceinline__ void tile_store(T* __restrict__ dst, const FrameLut& lut, uint64_t base, uint32_t nloc,
                                           const T* tile) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const uint32_t l = threadIdx.x + uint32_t(i) * NT;
    if (l < nloc) dst[base | frame_deposit(lut, l)] = tile[lds_swz(l)];
  }
}

// ---------------------------------------------------------------------------
// Full tiles (a frame of exactly B bits).  The frame-local index
// l = threadIdx.x + i NT has the thread's bits and the element's bits apart,
// and the frame map is a bit deposit, so l's global offset is thr | el(i):
// a per-thread part computed once and a part shared by the block.  No lookup
// table and no per-element guard: the loads of one tile leave back to back,
// and the compiler can count them instead of waiting for all memory traffic
// before each one.
// ---------------------------------------------------------------------------
constexpr int ilog2c(unsigned v) { return v <= 1u ? 0 : 1 + ilog2c(v >> 1); }

template <int NT, int PER>
struct TileAddr {
  static constexpr int kT = ilog2c(NT), kE = ilog2c(PER);
  uint64_t off[PER];  // thr | el(i), per thread (VGPRs; the uniform parts would hold SGPRs all kernel long)
  __device__ __forceinline__ explicit TileAddr(const FrameDesc& fr) {
    uint64_t thr = 0;
#pragma unroll
    for (int j = 0; j < kT; ++j) thr |= uint64_t((threadIdx.x >> j) & 1u) << fr.q[j];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      uint64_t g = thr;
#pragma unroll
      for (int k = 0; k < kE; ++k)
        if ((i >> k) & 1) g |= uint64_t(1) << fr.q[kT + k];
      off[i] = g;
    }
  }
};

// The same addressing with only the thread's part in registers (two VGPRs
// instead of 2 PER): the element's part comes from the frame, which the
// kernel holds in SGPRs, at each fetch.  For kernels whose work between the
// fetches needs the VGPRs.
template <int NT, int PER>
struct TileAddrLean {
  static constexpr int kT = ilog2c(NT), kE = ilog2c(PER);
  uint64_t thr;
  __device__ __forceinline__ explicit TileAddrLean(const FrameDesc& fr) {
    thr = 0;
#pragma unroll
    for (int j = 0; j < kT; ++j) thr |= uint64_t((threadIdx.x >> j) & 1u) << fr.q[j];
  }
};

// Offset of element i of the thread's share: the element's part is built on
// the scalar unit and made opaque to the optimiser, so it is recomputed at
// each use rather than hoisted out of the tile loop as PER 64-bit VGPR
// addresses.
template <int NT, int PER>
__device__ __forceinline__ uint64_t lean_off(const TileAddrLean<NT, PER>& a, const FrameDesc& fr, int i) {
  constexpr int kT = TileAddrLean<NT, PER>::kT, kE = TileAddrLean<NT, PER>::kE;
  uint64_t el = 0;  // uniform
#pragma unroll
  for (int k = 0; k < kE; ++k)
    if ((i >> k) & 1) el |= uint64_t(1) << fr.q[kT + k];
  uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(el)), hi = __builtin_amdgcn_readfirstlane(uint32_t(el >> 32));
  asm volatile("" : "+s"(lo), "+s"(hi));
  return a.thr | (uint64_t(hi) << 32 | lo);
}

template <typename T, int PER, int NT>
__device__ __forceinline__ void tile_fetch_full(const T* __restrict__ src, const TileAddrLean<NT, PER>& a,
                                                const FrameDesc& fr, uint64_t base, Stage<T, PER>& reg) {
  const T* p = src + base;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const T v = p[lean_off(a, fr, i)];
    reg.re[i] = v.x;
    reg.im[i] = v.y;
  }
}

template <typename T, int PER, int NT>
__device__ __forceinline__ void tile_send(T* __restrict__ dst, const TileAddrLean<NT, PER>& a, const FrameDesc& fr,
                                          uint64_t base, const Stage<T, PER>& reg) {
  T* p = dst + base;
#pragma unroll
  for (int i = 0; i < PER; ++i) p[lean_off(a, fr, i)] = cmake<T>(reg.re[i], reg.im[i]);
}

template <typename T, int PER, int NT>
__device__ __forceinline__ void tile_fetch_full(const T* __restrict__ src, const TileAddr<NT, PER>& a, uint64_t base,
                                                Stage<T, PER>& reg) {
  const T* p = src + base;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const T v = p[a.off[i]];
    reg.re[i] = v.x;
    reg.im[i] = v.y;
  }
}

template <typename T, int PER, int NT>
__device__ __forceinline__ void tile_put_full(T* tile, const Stage<T, PER>& reg) {
#pragma unroll
  for (int i = 0; i < PER; ++i) tile[lds_swz(threadIdx.x + uint32_t(i) * NT)] = cmake<T>(reg.re[i], reg.im[i]);
}

// The thread's own slots (the ones tile_put_full writes) into registers.
template <typename T, int PER, int NT>
__device__ __forceinline__ void tile_take(const T* tile, Stage<T, PER>& reg) {
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const T v = tile[lds_swz(threadIdx.x + uint32_t(i) * NT)];
    reg.re[i] = v.x;
    reg.im[i] = v.y;
  }
}

template <typename T, int PER, int NT>
__device__ __forceinline__ void tile_send(T* __restrict__ dst, const TileAddr<NT, PER>& a, uint64_t base,
                                          const Stage<T, PER>& reg) {
  T* p = dst + base;
#pragma unroll
  for (int i = 0; i < PER; ++i) p[a.off[i]] = cmake<T>(reg.re[i], reg.im[i]);
}

// ---------------------------------------------------------------------------
// fused-run pair arithmetic (Section 5.1, Eq. 11)
//
// For the pair (m, m' = m ^ x) with the pivot bit of m clear, the reference
// string acts as P0 psi[m] = beta psi[m'], P0 psi[m'] = conj(beta) psi[m] with
// beta = i^omega0 (-1)^{|m' & z0|}; every other string of the run is
// eps_k(m) P0 on the pair, so the run is exp(-i Phi P0 / 2) with
// Phi = sum_k eps_k phi_k, tabulated on the host as (cos Phi/2, sin Phi/2):
//   psi'[m]  = c psi[m]  - i s beta psi[m']
//   psi'[m'] = c psi[m'] - i s conj(beta) psi[m]
// The reverse sweep applies the inverse (s -> -s).
// ---------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ void rot_pair(V& a, V& b, typename Real<V>::type c, typename Real<V>::type s,
                                         unsigned sgn, unsigned omega0) {
  using R = typename Real<V>::type;
  const R ss = sgn ? -s : s;
  const V tb = mul_ipow(b, (omega0 + 3u) & 3u);
  const V ta = mul_ipow(a, (3u - omega0) & 3u);
  const V na = cmake<V>(c * a.x + ss * tb.x, c * a.y + ss * tb.y);
  const V nb = cmake<V>(c * b.x + ss * ta.x, c * b.y + ss * ta.y);
  a = na;
  b = nb;
}

// Gradient factor of a pair (Algorithm 1): dE/dphi_k = Im <lam|P_k|psi> sums
// eps_k(m) w over pairs, with
//   w = Im[conj(lam[m]) beta psi[m'] + conj(lam[m']) conj(beta) psi[m]]  (FP64)
template <typename V>
__device__ __forceinline__ double grad_w(V pa, V pb, V la, V lb, unsigned sgn, unsigned omega0) {
  if constexpr (is_real_amp<V>) {
    // real values and beta = +-i (omega0 odd; an even omega0 gives a
    // complex rotation, which a real state never takes): Im(beta) (la pb - lb pa)
    const double w = (double)la.x * (double)pb.x - (double)lb.x * (double)pa.x;
    const double v = (omega0 & 2u) ? -w : w;
    return ((omega0 & 1u) == 0u) ? 0.0 : (sgn ? -v : v);
  }
  const V tb = mul_ipow(pb, omega0 & 3u);
  const V ta = mul_ipow(pa, (4u - omega0) & 3u);
  double w = (double)la.x * (double)tb.y - (double)la.y * (double)tb.x + (double)lb.x * (double)ta.y -
             (double)lb.y * (double)ta.x;
  return sgn ? -w : w;
}

// The same two operations for a real rotation (omega0 = 1 or 3, omega = +-i)
// on a real pair, where every imaginary part is zero: rot_pair becomes
// a' = c a + q b, b' = c b - q a with q = +-s, and grad_w becomes
// +-(lam[m] psi[m'] - lam[m'] psi[m]).
template <unsigned OM, typename R>
__device__ __forceinline__ void rot_pair_real(R& a, R& b, R c, R s, unsigned sgn) {
  const R ss = sgn ? -s : s;
  const R q = OM == 1 ? ss : -ss;
  const R na = c * a + q * b;
  const R nb = c * b - q * a;
  a = na;
  b = nb;
}

template <unsigned OM, typename R>
__device__ __forceinline__ double grad_w_real(R pa, R pb, R la, R lb, unsigned sgn) {
  double w = (double)la * (double)pb - (double)lb * (double)pa;
  if (OM == 3) w = -w;
  return sgn ? -w : w;
}

// pattern index of m' (frame-local l2, block base) for kRunFull / kRunDiag
__device__ __forceinline__ unsigned run_pattern(const RunDesc& r, uint64_t l2, uint64_t base) {
  unsigned p = 0;
  for (int j = 0; j < r.n_pat; ++j) {
    const unsigned pos = pack_at(r.pat_pack, j);
    const uint64_t bit = pos < 64 ? (l2 >> pos) & 1ull : (base >> (pos - 64)) & 1ull;
    p |= unsigned(bit) << j;
  }
  return p;
}

}  // namespace q2sv
