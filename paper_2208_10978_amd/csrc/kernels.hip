// gfx950 kernels of the UCCSD state-vector path.
//
// Amplitudes are interleaved complex (double2 for complex128, float2 for
// complex64).  Sweeps compute in the amplitude precision; every reduction
// (energy, norm, gradient) promotes products to FP64 and sums them in a fixed
// order: per lane, then across the 64 lanes of a wavefront, then across the
// wavefronts of a block in index order, then across blocks in index order.
// No floating-point atomics are used, so results are bitwise reproducible.
//
// Pair update of a fused run (Section 5.1, Eq. 11).  For the pair
// (m, m' = m ^ x) with the pivot bit of m clear, the reference string acts as
// P0 psi[m] = beta psi[m'], P0 psi[m'] = conj(beta) psi[m] with
// beta = i^omega0 (-1)^{|m' & z0|}; every other string of the run is
// eps_k(m) P0 on the pair, so the run is exp(-i Phi P0 / 2) with
// Phi = sum_k eps_k phi_k, tabulated on the host as (cos Phi/2, sin Phi/2).
//   psi'[m]  = c psi[m]  - i s beta psi[m']
//   psi'[m'] = c psi[m'] - i s conj(beta) psi[m]
// The reverse sweep applies the inverse (s -> -s).
//
// Gradient (Algorithm 1).  dE/dphi_k = Im <lam|P_k|psi> with psi, lam taken
// right after the run.  Per pair the common factor is
//   w = Im[ conj(lam[m]) beta psi[m'] + conj(lam[m']) conj(beta) psi[m] ]
// and dE/dphi_k sums eps_k(m) w.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "q2sv_internal.h"

namespace q2sv {

template <typename T> struct Real;
template <> struct Real<double2> { using type = double; };
template <> struct Real<float2> { using type = float; };

template <typename V>
__device__ __forceinline__ V cmake(typename Real<V>::type re, typename Real<V>::type im) {
  V v; v.x = re; v.y = im; return v;
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

__device__ __forceinline__ uint64_t insert_zero(uint64_t t, unsigned pos) {
  const uint64_t low = t & ((uint64_t(1) << pos) - 1);
  return ((t >> pos) << (pos + 1)) | low;
}

// Insert zeros at ascending frame-local positions.
__device__ __forceinline__ uint64_t insert_zeros(uint64_t t, const uint8_t* pos, int n) {
  for (int j = 0; j < n; ++j) t = insert_zero(t, pos[j]);
  return t;
}

// ---------------------------------------------------------------------------
// deterministic block reduction of FP64 values
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
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
// frame helpers
// ---------------------------------------------------------------------------
struct FrameLut {
  // deposit of frame-local bits [c, c + k1) and [c + k1, B) to global positions
  uint64_t lo[128];
  uint64_t hi[128];
  int c, k1, b;
};

__device__ __forceinline__ uint64_t frame_base(const FrameDesc& fr, uint64_t tb) {
  uint64_t base = 0;
  for (int j = 0; j < fr.n_comp; ++j) base |= ((tb >> j) & 1ull) << fr.comp[j];
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
  if (threadIdx.x == 0) { lut.c = c; lut.k1 = k1; lut.b = b; }
}

__device__ __forceinline__ uint64_t frame_deposit(const FrameLut& lut, uint32_t l) {
  const uint32_t cm = (1u << lut.c) - 1u;
  const uint32_t m1 = (1u << lut.k1) - 1u;
  return uint64_t(l & cm) | lut.lo[(l >> lut.c) & m1] | lut.hi[l >> (lut.c + lut.k1)];
}

// pattern index of m' (frame-local l2, block base) for kRunFull / kRunDiag
__device__ __forceinline__ unsigned run_pattern(const RunDesc& r, uint64_t l2, uint64_t base) {
  unsigned p = 0;
  for (int j = 0; j < r.n_pat; ++j) {
    const unsigned pos = r.pat_pos[j];
    const uint64_t bit = pos < 64 ? (l2 >> pos) & 1ull : (base >> (pos - 64)) & 1ull;
    p |= unsigned(bit) << j;
  }
  return p;
}

// ---------------------------------------------------------------------------
// pair arithmetic
// ---------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ void rot_pair(V& a, V& b, typename Real<V>::type c, typename Real<V>::type s,
                                         unsigned sgn, unsigned omega0) {
  // a' = c a - i s beta b ;  b' = c b - i s conj(beta) a ;  beta = i^omega0 (-1)^sgn
  using R = typename Real<V>::type;
  const R ss = sgn ? -s : s;
  const V tb = mul_ipow(b, (omega0 + 3u) & 3u);
  const V ta = mul_ipow(a, (3u - omega0) & 3u);
  const V na = cmake<V>(c * a.x + ss * tb.x, c * a.y + ss * tb.y);
  const V nb = cmake<V>(c * b.x + ss * ta.x, c * b.y + ss * ta.y);
  a = na;
  b = nb;
}

// w = Im[conj(la) beta pb + conj(lb) conj(beta) pa], in FP64
template <typename V>
__device__ __forceinline__ double grad_w(V pa, V pb, V la, V lb, unsigned sgn, unsigned omega0) {
  const V tb = mul_ipow(pb, omega0 & 3u);
  const V ta = mul_ipow(pa, (4u - omega0) & 3u);
  // Im(conj(u) v) = u.x v.y - u.y v.x
  double w = (double)la.x * (double)tb.y - (double)la.y * (double)tb.x
           + (double)lb.x * (double)ta.y - (double)lb.y * (double)ta.x;
  return sgn ? -w : w;
}

// ---------------------------------------------------------------------------
// HF preparation (Eq. 6): psi = |k>
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_fill_basis(T* psi, uint64_t n_amp, uint64_t k) {
  using R = typename Real<T>::type;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_amp; i += stride)
    psi[i] = cmake<T>(i == k ? R(1) : R(0), R(0));
}

// ---------------------------------------------------------------------------
// one run over the whole state (identity frame)
// GRAD: 0 none (forward), 1 per-run parameter gradient, 2 per-string gradient
// ---------------------------------------------------------------------------
template <typename T, bool REV, int GRAD>
__global__ void __launch_bounds__(256) k_run_full(T* __restrict__ psi, T* __restrict__ lam, RunDesc run,
                                                  const RunRec* __restrict__ recs, double* __restrict__ partials,
                                                  int n, uint32_t nb_stride) {
  using R = typename Real<T>::type;
  __shared__ double red[4];
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  const uint64_t tid0 = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  double acc[GRAD == 2 ? kMaxRunStrings : 1];
#pragma unroll
  for (int k = 0; k < (GRAD == 2 ? kMaxRunStrings : 1); ++k) acc[k] = 0.0;

  if (run.mode == kRunEnum) {
    const uint64_t npairs = uint64_t(1) << (n - run.n_sup);
    for (int r = 0; r < run.n_rec; ++r) {
      const RunRec rec = recs[run.rec_off + r];
      const R c = R(rec.c), s = REV ? R(-rec.s) : R(rec.s);
      double wsum = 0.0;
      for (uint64_t t = tid0; t < npairs; t += stride) {
        const uint64_t m2 = insert_zeros(t, run.sup_pos, run.n_sup) | rec.bits;
        const uint64_t m = m2 ^ run.x_loc;
        const unsigned sg = parity64(m2 & run.z0_loc);
        T a = psi[m], b = psi[m2];
        if (GRAD) {
          const T la = lam[m], lb = lam[m2];
          wsum += grad_w(a, b, la, lb, sg, run.omega0);
          T la2 = la, lb2 = lb;
          rot_pair(la2, lb2, c, s, sg, run.omega0);
          lam[m] = la2; lam[m2] = lb2;
        }
        rot_pair(a, b, c, s, sg, run.omega0);
        psi[m] = a; psi[m2] = b;
      }
      if (GRAD == 1) acc[0] += rec.a * wsum;
      if (GRAD == 2) {
#pragma unroll
        for (int k = 0; k < kMaxRunStrings; ++k)
          acc[k] += ((rec.eps_neg >> k) & 1u) ? -wsum : wsum;
      }
    }
  } else if (run.mode == kRunFull) {
    const uint64_t npairs = uint64_t(1) << (n - 1);
    for (uint64_t t = tid0; t < npairs; t += stride) {
      const uint64_t m = insert_zero(t, run.pivot);
      const uint64_t m2 = m ^ run.x_loc;
      const unsigned sg = parity64(m2 & run.z0_loc);
      const unsigned p = run_pattern(run, m2, 0);
      const RunRec rec = recs[run.rec_off + p];
      const R c = R(rec.c), s = REV ? R(-rec.s) : R(rec.s);
      T a = psi[m], b = psi[m2];
      if (GRAD) {
        const T la = lam[m], lb = lam[m2];
        const double w = grad_w(a, b, la, lb, sg, run.omega0);
        if (GRAD == 1) acc[0] += rec.a * w;
        if (GRAD == 2) {
#pragma unroll
          for (int k = 0; k < kMaxRunStrings; ++k) {
            const unsigned e = ((run.str_neg >> k) & 1u) ^ (__popc(p & run.str_dpat[k]) & 1u);
            acc[k] += e ? -w : w;
          }
        }
        T la2 = la, lb2 = lb;
        rot_pair(la2, lb2, c, s, sg, run.omega0);
        lam[m] = la2; lam[m2] = lb2;
      }
      rot_pair(a, b, c, s, sg, run.omega0);
      psi[m] = a; psi[m2] = b;
    }
  } else {  // kRunDiag: psi[m] <- (c - i s (-1)^{|m & z0|}) psi[m]
    const uint64_t n_amp = uint64_t(1) << n;
    for (uint64_t m = tid0; m < n_amp; m += stride) {
      const unsigned sg = parity64(m & run.z0_loc);
      const unsigned p = run_pattern(run, m, 0);
      const RunRec rec = recs[run.rec_off + p];
      const R c = R(rec.c);
      const R s = (REV ? R(-rec.s) : R(rec.s)) * (sg ? R(-1) : R(1));
      T a = psi[m];
      if (GRAD) {
        const T la = lam[m];
        // Im(conj(la) (-1)^sg a)
        double w = (double)la.x * (double)a.y - (double)la.y * (double)a.x;
        if (sg) w = -w;
        if (GRAD == 1) acc[0] += rec.a * w;
        if (GRAD == 2) {
#pragma unroll
          for (int k = 0; k < kMaxRunStrings; ++k) {
            const unsigned e = ((run.str_neg >> k) & 1u) ^ (__popc(p & run.str_dpat[k]) & 1u);
            acc[k] += e ? -w : w;
          }
        }
        lam[m] = cmake<T>(c * la.x + s * la.y, c * la.y - s * la.x);
      }
      psi[m] = cmake<T>(c * a.x + s * a.y, c * a.y - s * a.x);
    }
  }
  if (GRAD) {
    const int nk = GRAD == 2 ? run.n_str : 1;
    for (int k = 0; k < (GRAD == 2 ? kMaxRunStrings : 1); ++k) {
      if (k >= nk) break;
      const double v = block_sum<256>(acc[k], red);
      if (threadIdx.x == 0) partials[uint64_t(run.slot + k) * nb_stride + blockIdx.x] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// LDS tile: load, apply every run of the pass, store.  Forward only.
// ---------------------------------------------------------------------------
template <typename T, int B, int NT>
__global__ void __launch_bounds__(NT) k_tile_forward(T* __restrict__ psi, FrameDesc fr,
                                                     const RunDesc* __restrict__ runs, int n_runs,
                                                     const RunRec* __restrict__ recs, uint64_t n_tb) {
  using R = typename Real<T>::type;
  __shared__ T tile[1 << B];
  __shared__ FrameLut lut;
  frame_lut_init<NT>(fr, lut);
  __syncthreads();
  const uint32_t nloc = 1u << fr.b;
  for (uint64_t tb = blockIdx.x; tb < n_tb; tb += gridDim.x) {
    const uint64_t base = frame_base(fr, tb);
    for (uint32_t l = threadIdx.x; l < nloc; l += NT) tile[l] = psi[base | frame_deposit(lut, l)];
    __syncthreads();
    for (int ri = 0; ri < n_runs; ++ri) {
      const RunDesc run = runs[ri];
      const unsigned so = parity64(base & run.z0_out);
      if (run.mode == kRunEnum) {
        const uint32_t np = nloc >> run.n_sup;
        for (int r = 0; r < run.n_rec; ++r) {
          const RunRec rec = recs[run.rec_off + r];
          const R c = R(rec.c), s = R(rec.s);
          for (uint32_t t = threadIdx.x; t < np; t += NT) {
            const uint32_t l2 = uint32_t(insert_zeros(t, run.sup_pos, run.n_sup) | rec.bits);
            const uint32_t l = l2 ^ uint32_t(run.x_loc);
            const unsigned sg = so ^ (__popc(l2 & uint32_t(run.z0_loc)) & 1u);
            T a = tile[l], b = tile[l2];
            rot_pair(a, b, c, s, sg, run.omega0);
            tile[l] = a; tile[l2] = b;
          }
        }
      } else if (run.mode == kRunFull) {
        const uint32_t np = nloc >> 1;
        for (uint32_t t = threadIdx.x; t < np; t += NT) {
          const uint32_t l = uint32_t(insert_zero(t, run.pivot));
          const uint32_t l2 = l ^ uint32_t(run.x_loc);
          const unsigned sg = so ^ (__popc(l2 & uint32_t(run.z0_loc)) & 1u);
          const RunRec rec = recs[run.rec_off + run_pattern(run, l2, base)];
          T a = tile[l], b = tile[l2];
          rot_pair(a, b, R(rec.c), R(rec.s), sg, run.omega0);
          tile[l] = a; tile[l2] = b;
        }
      } else {
        for (uint32_t l = threadIdx.x; l < nloc; l += NT) {
          const unsigned sg = so ^ (__popc(l & uint32_t(run.z0_loc)) & 1u);
          const RunRec rec = recs[run.rec_off + run_pattern(run, l, base)];
          const R c = R(rec.c), s = R(rec.s) * (sg ? R(-1) : R(1));
          const T a = tile[l];
          tile[l] = cmake<T>(c * a.x + s * a.y, c * a.y - s * a.x);
        }
      }
      __syncthreads();
    }
    for (uint32_t l = threadIdx.x; l < nloc; l += NT) psi[base | frame_deposit(lut, l)] = tile[l];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// LDS tile, reverse sweep: psi and lam tiles; for every run of the pass (in
// pass order, which is reverse list order) accumulate the gradient factor and
// undo the run on both.  Gradient partials per local slot are summed per
// wavefront into LDS, then written once per block.
// ---------------------------------------------------------------------------
template <int NT, int MAXS>
struct GradAcc { double v[MAXS][NT / 64]; };

template <typename T, int B, int NT, int GRAD, int MAXS>
__global__ void __launch_bounds__(NT) k_tile_reverse(T* __restrict__ psi, T* __restrict__ lam, FrameDesc fr,
                                                     const RunDesc* __restrict__ runs, int n_runs,
                                                     const RunRec* __restrict__ recs,
                                                     const uint32_t* __restrict__ slot_map, int n_slots,
                                                     double* __restrict__ partials, uint32_t nb_stride,
                                                     uint64_t n_tb) {
  using R = typename Real<T>::type;
  constexpr int NW = NT / 64;
  __shared__ T tp[1 << B];
  __shared__ T tl[1 << B];
  __shared__ FrameLut lut;
  __shared__ GradAcc<NT, MAXS> gacc;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  frame_lut_init<NT>(fr, lut);
  for (int i = threadIdx.x; i < MAXS * NW; i += NT) (&gacc.v[0][0])[i] = 0.0;
  __syncthreads();
  const uint32_t nloc = 1u << fr.b;
  for (uint64_t tb = blockIdx.x; tb < n_tb; tb += gridDim.x) {
    const uint64_t base = frame_base(fr, tb);
    for (uint32_t l = threadIdx.x; l < nloc; l += NT) {
      const uint64_t g = base | frame_deposit(lut, l);
      tp[l] = psi[g];
      tl[l] = lam[g];
    }
    __syncthreads();
    for (int ri = 0; ri < n_runs; ++ri) {
      const RunDesc run = runs[ri];
      const unsigned so = parity64(base & run.z0_out);
      double acc[GRAD == 2 ? kMaxRunStrings : 1];
#pragma unroll
      for (int k = 0; k < (GRAD == 2 ? kMaxRunStrings : 1); ++k) acc[k] = 0.0;
      if (run.mode == kRunEnum) {
        const uint32_t np = nloc >> run.n_sup;
        for (int r = 0; r < run.n_rec; ++r) {
          const RunRec rec = recs[run.rec_off + r];
          const R c = R(rec.c), s = R(-rec.s);
          double wsum = 0.0;
          for (uint32_t t = threadIdx.x; t < np; t += NT) {
            const uint32_t l2 = uint32_t(insert_zeros(t, run.sup_pos, run.n_sup) | rec.bits);
            const uint32_t l = l2 ^ uint32_t(run.x_loc);
            const unsigned sg = so ^ (__popc(l2 & uint32_t(run.z0_loc)) & 1u);
            T a = tp[l], b = tp[l2], la = tl[l], lb = tl[l2];
            if (GRAD) wsum += grad_w(a, b, la, lb, sg, run.omega0);
            rot_pair(a, b, c, s, sg, run.omega0);
            rot_pair(la, lb, c, s, sg, run.omega0);
            tp[l] = a; tp[l2] = b; tl[l] = la; tl[l2] = lb;
          }
          if (GRAD == 1) acc[0] += rec.a * wsum;
          if (GRAD == 2) {
#pragma unroll
            for (int k = 0; k < kMaxRunStrings; ++k) acc[k] += ((rec.eps_neg >> k) & 1u) ? -wsum : wsum;
          }
        }
      } else if (run.mode == kRunFull) {
        const uint32_t np = nloc >> 1;
        for (uint32_t t = threadIdx.x; t < np; t += NT) {
          const uint32_t l = uint32_t(insert_zero(t, run.pivot));
          const uint32_t l2 = l ^ uint32_t(run.x_loc);
          const unsigned sg = so ^ (__popc(l2 & uint32_t(run.z0_loc)) & 1u);
          const unsigned p = run_pattern(run, l2, base);
          const RunRec rec = recs[run.rec_off + p];
          T a = tp[l], b = tp[l2], la = tl[l], lb = tl[l2];
          if (GRAD) {
            const double w = grad_w(a, b, la, lb, sg, run.omega0);
            if (GRAD == 1) acc[0] += rec.a * w;
            if (GRAD == 2) {
#pragma unroll
              for (int k = 0; k < kMaxRunStrings; ++k) {
                const unsigned e = ((run.str_neg >> k) & 1u) ^ (__popc(p & run.str_dpat[k]) & 1u);
                acc[k] += e ? -w : w;
              }
            }
          }
          rot_pair(a, b, R(rec.c), R(-rec.s), sg, run.omega0);
          rot_pair(la, lb, R(rec.c), R(-rec.s), sg, run.omega0);
          tp[l] = a; tp[l2] = b; tl[l] = la; tl[l2] = lb;
        }
      } else {
        for (uint32_t l = threadIdx.x; l < nloc; l += NT) {
          const unsigned sg = so ^ (__popc(l & uint32_t(run.z0_loc)) & 1u);
          const unsigned p = run_pattern(run, l, base);
          const RunRec rec = recs[run.rec_off + p];
          const T a = tp[l], la = tl[l];
          if (GRAD) {
            double w = (double)la.x * (double)a.y - (double)la.y * (double)a.x;
            if (sg) w = -w;
            if (GRAD == 1) acc[0] += rec.a * w;
            if (GRAD == 2) {
#pragma unroll
              for (int k = 0; k < kMaxRunStrings; ++k) {
                const unsigned e = ((run.str_neg >> k) & 1u) ^ (__popc(p & run.str_dpat[k]) & 1u);
                acc[k] += e ? -w : w;
              }
            }
          }
          const R c = R(rec.c), s = R(-rec.s) * (sg ? R(-1) : R(1));
          tp[l] = cmake<T>(c * a.x + s * a.y, c * a.y - s * a.x);
          tl[l] = cmake<T>(c * la.x + s * la.y, c * la.y - s * la.x);
        }
      }
      if (GRAD) {
        const int nk = GRAD == 2 ? run.n_str : 1;
        for (int k = 0; k < (GRAD == 2 ? kMaxRunStrings : 1); ++k) {
          if (k >= nk) break;
          const double v = wave_sum(acc[k]);
          if (lane == 0) gacc.v[run.slot + k][wave] += v;
        }
      }
      __syncthreads();
    }
    for (uint32_t l = threadIdx.x; l < nloc; l += NT) {
      const uint64_t g = base | frame_deposit(lut, l);
      psi[g] = tp[l];
      lam[g] = tl[l];
    }
    __syncthreads();
  }
  if (GRAD) {
    for (int i = threadIdx.x; i < n_slots; i += NT) {
      double s = 0.0;
      for (int w = 0; w < NW; ++w) s += gacc.v[i][w];
      partials[uint64_t(slot_map[i]) * nb_stride + blockIdx.x] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Pauli-sum groups over an LDS tile.
//   MODE 0: expectation partials  sum_m conj(psi[m]) (H_x psi)[m]  (real part)
//   MODE 1: lam  = sum over the tile's groups of H_x psi   (first pass)
//   MODE 2: lam += sum over the tile's groups of H_x psi
// For MODE 0 the launch covers several tiles: block b works on tile
// tile_first + b / blocks_per_tile.
// ---------------------------------------------------------------------------
template <typename T, int B, int NT, int MODE>
__global__ void __launch_bounds__(NT) k_tile_hamiltonian(
    const T* __restrict__ psi, T* __restrict__ lam, const FrameDesc* __restrict__ frames,
    const uint32_t* __restrict__ tile_groups,  // [tile] -> first group; tile_groups[tile+1] end
    const GroupDesc* __restrict__ groups, const SubDesc* __restrict__ subs,
    const double2* __restrict__ coef, const uint64_t* __restrict__ recbits, int tile_first,
    uint32_t blocks_per_tile, uint64_t n_tb, double* __restrict__ partials) {
  using R = typename Real<T>::type;
  __shared__ T tp[1 << B];
  __shared__ T tl[MODE == 0 ? 1 : (1 << B)];
  __shared__ FrameLut lut;
  __shared__ double red[NT / 64];
  const int tile = tile_first + int(blockIdx.x / blocks_per_tile);
  const uint32_t bi = blockIdx.x % blocks_per_tile;
  const FrameDesc fr = frames[tile];
  frame_lut_init<NT>(fr, lut);
  __syncthreads();
  const uint32_t nloc = 1u << fr.b;
  const uint32_t g0 = tile_groups[tile], g1 = tile_groups[tile + 1];
  double e = 0.0;
  for (uint64_t tb = bi; tb < n_tb; tb += blocks_per_tile) {
    const uint64_t base = frame_base(fr, tb);
    for (uint32_t l = threadIdx.x; l < nloc; l += NT) {
      tp[l] = psi[base | frame_deposit(lut, l)];
      if (MODE != 0) tl[l] = cmake<T>(R(0), R(0));
    }
    __syncthreads();
    for (uint32_t gi = g0; gi < g1; ++gi) {
      const GroupDesc g = groups[gi];
      if (g.is_diag) {
        for (uint32_t l = threadIdx.x; l < nloc; l += NT) {
          double gre = 0.0, gim = 0.0;
          for (uint32_t k = 0; k < g.n_sub; ++k) {
            const SubDesc sd = subs[g.sub_off + k];
            const double2 cv = coef[sd.coef_off];
            const unsigned sg = parity64(base & sd.w_out) ^ (__popc(l & uint32_t(sd.w_loc)) & 1u);
            gre += sg ? -cv.x : cv.x;
            gim += sg ? -cv.y : cv.y;
          }
          const T a = tp[l];
          if (MODE == 0) {
            e += gre * ((double)a.x * a.x + (double)a.y * a.y);
          } else {
            T v = tl[l];
            v.x += R(gre * a.x - gim * a.y);
            v.y += R(gre * a.y + gim * a.x);
            tl[l] = v;
          }
        }
      } else {
        const uint32_t np = g.enumerated ? (nloc >> g.n_sup) : (nloc >> 1);
        for (int r = 0; r < g.n_rec; ++r) {
          const uint32_t bits = g.enumerated ? uint32_t(recbits[g.rec_off + r]) : 0u;
          for (uint32_t t = threadIdx.x; t < np; t += NT) {
            uint32_t l2, l;
            if (g.enumerated) {
              l2 = uint32_t(insert_zeros(t, g.sup_pos, g.n_sup)) | bits;
              l = l2 ^ uint32_t(g.x_loc);
            } else {
              l = uint32_t(insert_zero(t, g.pivot));
              l2 = l ^ uint32_t(g.x_loc);
            }
            double gre = 0.0, gim = 0.0;
            for (uint32_t k = 0; k < g.n_sub; ++k) {
              const SubDesc sd = subs[g.sub_off + k];
              const double2 cv = coef[sd.coef_off + r];
              const unsigned sg = parity64(base & sd.w_out) ^ (__popc(l2 & uint32_t(sd.w_loc)) & 1u);
              gre += sg ? -cv.x : cv.x;
              gim += sg ? -cv.y : cv.y;
            }
            const T a = tp[l], b = tp[l2];
            if (MODE == 0) {
              // 2 Re(conj(a) G b)
              const double gbr = gre * b.x - gim * b.y, gbi = gre * b.y + gim * b.x;
              e += 2.0 * ((double)a.x * gbr + (double)a.y * gbi);
            } else {
              // lam[l] += G b ; lam[l2] += conj(G) a
              T u = tl[l], v = tl[l2];
              u.x += R(gre * b.x - gim * b.y);
              u.y += R(gre * b.y + gim * b.x);
              v.x += R(gre * a.x + gim * a.y);
              v.y += R(gre * a.y - gim * a.x);
              tl[l] = u;
              tl[l2] = v;
            }
          }
        }
      }
      if (MODE != 0) __syncthreads();
    }
    if (MODE != 0) {
      for (uint32_t l = threadIdx.x; l < nloc; l += NT) {
        const uint64_t gidx = base | frame_deposit(lut, l);
        T v = tl[l];
        if (MODE == 2) {
          const T o = lam[gidx];
          v.x += o.x;
          v.y += o.y;
        }
        lam[gidx] = v;
      }
    }
    __syncthreads();
  }
  if (MODE == 0) {
    const double s = block_sum<NT>(e, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// one group over the whole state (groups whose support does not fit a tile)
// MODE as above; lam updated in place in global memory.
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_group_full(const T* __restrict__ psi, T* __restrict__ lam,
                                                    GroupDesc g, const SubDesc* __restrict__ subs,
                                                    const double2* __restrict__ coef,
                                                    const uint64_t* __restrict__ recbits, int n,
                                                    double* __restrict__ partials) {
  using R = typename Real<T>::type;
  __shared__ double red[4];
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  const uint64_t tid0 = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  double e = 0.0;
  if (g.is_diag) {
    const uint64_t n_amp = uint64_t(1) << n;
    for (uint64_t m = tid0; m < n_amp; m += stride) {
      double gre = 0.0, gim = 0.0;
      for (uint32_t k = 0; k < g.n_sub; ++k) {
        const SubDesc sd = subs[g.sub_off + k];
        const double2 cv = coef[sd.coef_off];
        const unsigned sg = parity64(m & sd.w_loc);
        gre += sg ? -cv.x : cv.x;
        gim += sg ? -cv.y : cv.y;
      }
      const T a = psi[m];
      if (MODE == 0) {
        e += gre * ((double)a.x * a.x + (double)a.y * a.y);
      } else {
        T v = MODE == 1 ? cmake<T>(R(0), R(0)) : lam[m];
        v.x += R(gre * a.x - gim * a.y);
        v.y += R(gre * a.y + gim * a.x);
        lam[m] = v;
      }
    }
  } else {
    const uint64_t np = g.enumerated ? (uint64_t(1) << (n - g.n_sup)) : (uint64_t(1) << (n - 1));
    for (int r = 0; r < g.n_rec; ++r) {
      const uint64_t bits = g.enumerated ? recbits[g.rec_off + r] : 0ull;
      for (uint64_t t = tid0; t < np; t += stride) {
        uint64_t l2, l;
        if (g.enumerated) {
          l2 = insert_zeros(t, g.sup_pos, g.n_sup) | bits;
          l = l2 ^ g.x_loc;
        } else {
          l = insert_zero(t, g.pivot);
          l2 = l ^ g.x_loc;
        }
        double gre = 0.0, gim = 0.0;
        for (uint32_t k = 0; k < g.n_sub; ++k) {
          const SubDesc sd = subs[g.sub_off + k];
          const double2 cv = coef[sd.coef_off + r];
          const unsigned sg = parity64(l2 & sd.w_loc);
          gre += sg ? -cv.x : cv.x;
          gim += sg ? -cv.y : cv.y;
        }
        const T a = psi[l], b = psi[l2];
        if (MODE == 0) {
          const double gbr = gre * b.x - gim * b.y, gbi = gre * b.y + gim * b.x;
          e += 2.0 * ((double)a.x * gbr + (double)a.y * gbi);
        } else {
          T u = MODE == 1 ? cmake<T>(R(0), R(0)) : lam[l];
          T v = MODE == 1 ? cmake<T>(R(0), R(0)) : lam[l2];
          u.x += R(gre * b.x - gim * b.y);
          u.y += R(gre * b.y + gim * b.x);
          v.x += R(gre * a.x + gim * a.y);
          v.y += R(gre * a.y - gim * a.x);
          lam[l] = u;
          lam[l2] = v;
        }
      }
    }
  }
  if (MODE == 0) {
    const double s = block_sum<256>(e, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// reductions and small utilities
// ---------------------------------------------------------------------------

// partials[0][b] = sum conj(a)·b (real part) over the block, partials[1][b] = sum |a|^2
template <typename T>
__global__ void __launch_bounds__(256) k_dot(const T* __restrict__ a, const T* __restrict__ b, uint64_t n_amp,
                                             double* __restrict__ partials) {
  __shared__ double red[4];
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  double re = 0.0, nn = 0.0;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n_amp; i += stride) {
    const T u = a[i];
    nn += (double)u.x * u.x + (double)u.y * u.y;
    if (b) {
      const T v = b[i];
      re += (double)u.x * v.x + (double)u.y * v.y;
    }
  }
  const double s0 = block_sum<256>(re, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s0;
  const double s1 = block_sum<256>(nn, red);
  if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = s1;
}

// out[row] = sum_{j < len} in[row * stride + j], fixed order (one block per row)
__global__ void __launch_bounds__(256) k_reduce_rows(const double* __restrict__ in, uint64_t stride, uint32_t len,
                                                     double* __restrict__ out) {
  __shared__ double red[4];
  const uint64_t row = blockIdx.x;
  double s = 0.0;
  for (uint32_t j = threadIdx.x; j < len; j += 256) s += in[row * stride + j];
  const double t = block_sum<256>(s, red);
  if (threadIdx.x == 0) out[row] = t;
}

// out[0] = (sum_j h[j]) / norm, out[1] = norm, from reduced sums h[0..nh) and norm
__global__ void k_finish_energy(const double* __restrict__ sums, int nh, const double* __restrict__ norm,
                                double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double e = 0.0;
    for (int j = 0; j < nh; ++j) e += sums[j];
    const double nn = norm[0];
    out[0] = e / nn;
    out[1] = nn;
  }
}

// grad[i] = sum over the slots listed for output i, in list order
__global__ void __launch_bounds__(256) k_gather_slots(const double* __restrict__ slot_val,
                                                      const uint32_t* __restrict__ off,
                                                      const uint32_t* __restrict__ idx,
                                                      const double* __restrict__ weight, int n_out,
                                                      double* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_out) return;
  double s = 0.0;
  for (uint32_t k = off[i]; k < off[i + 1]; ++k) s += weight[k] * slot_val[idx[k]];
  out[i] = s;
}

__global__ void __launch_bounds__(256) k_fill_f64(double* __restrict__ p, uint64_t n, double v) {
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <typename T>
__global__ void __launch_bounds__(256) k_scale(T* __restrict__ psi, uint64_t n_amp, const double* __restrict__ norm2) {
  using R = typename Real<T>::type;
  const R f = R(1.0 / sqrt(norm2[0]));
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  for (uint64_t i = uint64_t(blockIdx.x) * 256 + threadIdx.x; i < n_amp; i += stride) {
    T v = psi[i];
    v.x *= f;
    v.y *= f;
    psi[i] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_gather_amps(const T* __restrict__ psi, const uint64_t* __restrict__ idx,
                                                     int64_t count, double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= count) return;
  const T v = psi[idx[i]];
  out[2 * i] = v.x;
  out[2 * i + 1] = v.y;
}

}  // namespace q2sv

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#include "launch.h"

namespace q2sv {

template <typename T>
static hipError_t run_full_t(bool rev, int grad, void* psi, void* lam, const RunDesc& run, const RunRec* recs,
                             double* partials, int n, uint32_t nb, int grid, hipStream_t st) {
  T* p = static_cast<T*>(psi);
  T* l = static_cast<T*>(lam);
  if (!rev) {
    hipLaunchKernelGGL((k_run_full<T, false, 0>), dim3(grid), dim3(256), 0, st, p, l, run, recs, partials, n, nb);
  } else if (grad == 0) {
    hipLaunchKernelGGL((k_run_full<T, true, 0>), dim3(grid), dim3(256), 0, st, p, l, run, recs, partials, n, nb);
  } else if (grad == 1) {
    hipLaunchKernelGGL((k_run_full<T, true, 1>), dim3(grid), dim3(256), 0, st, p, l, run, recs, partials, n, nb);
  } else {
    hipLaunchKernelGGL((k_run_full<T, true, 2>), dim3(grid), dim3(256), 0, st, p, l, run, recs, partials, n, nb);
  }
  return hipGetLastError();
}

hipError_t launch_fill_basis(int dtype, void* psi, uint64_t n_amp, uint64_t k, hipStream_t st) {
  const uint64_t want = (n_amp + 255) / 256;
  const int grid = int(want < 4096 ? (want ? want : 1) : 4096);
  if (dtype == 0)
    hipLaunchKernelGGL((k_fill_basis<double2>), dim3(grid), dim3(256), 0, st, static_cast<double2*>(psi), n_amp, k);
  else
    hipLaunchKernelGGL((k_fill_basis<float2>), dim3(grid), dim3(256), 0, st, static_cast<float2*>(psi), n_amp, k);
  return hipGetLastError();
}

hipError_t launch_run_full(int dtype, bool rev, int grad, void* psi, void* lam, const RunDesc& run,
                           const RunRec* recs, double* partials, int n, uint32_t nb_stride, int grid,
                           hipStream_t st) {
  if (dtype == 0) return run_full_t<double2>(rev, grad, psi, lam, run, recs, partials, n, nb_stride, grid, st);
  return run_full_t<float2>(rev, grad, psi, lam, run, recs, partials, n, nb_stride, grid, st);
}

hipError_t launch_tile_forward(int dtype, void* psi, const FrameDesc& fr, const RunDesc* runs, int n_runs,
                               const RunRec* recs, uint64_t n_tb, int grid, hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL((k_tile_forward<double2, kTileFwdC128, kTileThreads>), dim3(grid), dim3(kTileThreads), 0,
                       st, static_cast<double2*>(psi), fr, runs, n_runs, recs, n_tb);
  else
    hipLaunchKernelGGL((k_tile_forward<float2, kTileFwdC64, kTileThreads>), dim3(grid), dim3(kTileThreads), 0,
                       st, static_cast<float2*>(psi), fr, runs, n_runs, recs, n_tb);
  return hipGetLastError();
}

template <typename T, int B>
static hipError_t tile_reverse_t(int grad, void* psi, void* lam, const FrameDesc& fr, const RunDesc* runs,
                                 int n_runs, const RunRec* recs, const uint32_t* slot_map, int n_slots,
                                 double* partials, uint32_t nb, uint64_t n_tb, int grid, hipStream_t st) {
  T* p = static_cast<T*>(psi);
  T* l = static_cast<T*>(lam);
  if (grad == 0)
    hipLaunchKernelGGL((k_tile_reverse<T, B, kTileThreads, 0, 1>), dim3(grid), dim3(kTileThreads), 0, st, p, l,
                       fr, runs, n_runs, recs, slot_map, n_slots, partials, nb, n_tb);
  else if (grad == 1)
    hipLaunchKernelGGL((k_tile_reverse<T, B, kTileThreads, 1, kMaxPassSlots>), dim3(grid), dim3(kTileThreads), 0,
                       st, p, l, fr, runs, n_runs, recs, slot_map, n_slots, partials, nb, n_tb);
  else
    hipLaunchKernelGGL((k_tile_reverse<T, B, kTileThreads, 2, kMaxPassSlots>), dim3(grid), dim3(kTileThreads), 0,
                       st, p, l, fr, runs, n_runs, recs, slot_map, n_slots, partials, nb, n_tb);
  return hipGetLastError();
}

hipError_t launch_tile_reverse(int dtype, int grad, void* psi, void* lam, const FrameDesc& fr,
                               const RunDesc* runs, int n_runs, const RunRec* recs,
                               const uint32_t* slot_map, int n_slots, double* partials, uint32_t nb_stride,
                               uint64_t n_tb, int grid, hipStream_t st) {
  if (dtype == 0)
    return tile_reverse_t<double2, kTileTwoC128>(grad, psi, lam, fr, runs, n_runs, recs, slot_map, n_slots,
                                                 partials, nb_stride, n_tb, grid, st);
  return tile_reverse_t<float2, kTileTwoC64>(grad, psi, lam, fr, runs, n_runs, recs, slot_map, n_slots, partials,
                                             nb_stride, n_tb, grid, st);
}

template <typename T, int B, int MODE>
static void tile_h_t(const void* psi, void* lam, const FrameDesc* frames, const uint32_t* tg, const GroupDesc* g,
                     const SubDesc* s, const double2* c, const uint64_t* rb, int tf, int ntl, uint32_t bpt,
                     uint64_t n_tb, double* part, hipStream_t st) {
  hipLaunchKernelGGL((k_tile_hamiltonian<T, B, kTileThreads, MODE>), dim3(uint32_t(ntl) * bpt),
                     dim3(kTileThreads), 0, st, static_cast<const T*>(psi), static_cast<T*>(lam), frames, tg, g,
                     s, c, rb, tf, bpt, n_tb, part);
}

hipError_t launch_tile_hamiltonian(int dtype, int mode, const void* psi, void* lam, const FrameDesc* frames,
                                   const uint32_t* tile_groups, const GroupDesc* groups, const SubDesc* subs,
                                   const double2* coef, const uint64_t* recbits, int tile_first,
                                   int n_tiles_launch, uint32_t bpt, uint64_t n_tb, double* partials,
                                   hipStream_t st) {
#define Q2SV_TH(T, B, M) tile_h_t<T, B, M>(psi, lam, frames, tile_groups, groups, subs, coef, recbits, \
                                           tile_first, n_tiles_launch, bpt, n_tb, partials, st)
  if (dtype == 0) {
    if (mode == 0) Q2SV_TH(double2, kTileFwdC128, 0);
    else if (mode == 1) Q2SV_TH(double2, kTileTwoC128, 1);
    else Q2SV_TH(double2, kTileTwoC128, 2);
  } else {
    if (mode == 0) Q2SV_TH(float2, kTileFwdC64, 0);
    else if (mode == 1) Q2SV_TH(float2, kTileTwoC64, 1);
    else Q2SV_TH(float2, kTileTwoC64, 2);
  }
#undef Q2SV_TH
  return hipGetLastError();
}

hipError_t launch_group_full(int dtype, int mode, const void* psi, void* lam, const GroupDesc& g,
                             const SubDesc* subs, const double2* coef, const uint64_t* recbits, int n, int grid,
                             double* partials, hipStream_t st) {
#define Q2SV_GF(T, M)                                                                                  \
  hipLaunchKernelGGL((k_group_full<T, M>), dim3(grid), dim3(256), 0, st, static_cast<const T*>(psi), \
                     static_cast<T*>(lam), g, subs, coef, recbits, n, partials)
  if (dtype == 0) {
    if (mode == 0) Q2SV_GF(double2, 0);
    else if (mode == 1) Q2SV_GF(double2, 1);
    else Q2SV_GF(double2, 2);
  } else {
    if (mode == 0) Q2SV_GF(float2, 0);
    else if (mode == 1) Q2SV_GF(float2, 1);
    else Q2SV_GF(float2, 2);
  }
#undef Q2SV_GF
  return hipGetLastError();
}

hipError_t launch_dot(int dtype, const void* a, const void* b, uint64_t n_amp, int grid, double* partials,
                      hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL((k_dot<double2>), dim3(grid), dim3(256), 0, st, static_cast<const double2*>(a),
                       static_cast<const double2*>(b), n_amp, partials);
  else
    hipLaunchKernelGGL((k_dot<float2>), dim3(grid), dim3(256), 0, st, static_cast<const float2*>(a),
                       static_cast<const float2*>(b), n_amp, partials);
  return hipGetLastError();
}

hipError_t launch_reduce_rows(const double* in, uint64_t stride, uint32_t len, uint32_t rows, double* out,
                              hipStream_t st) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_rows, dim3(rows), dim3(256), 0, st, in, stride, len, out);
  return hipGetLastError();
}

hipError_t launch_finish_energy(const double* sums, int nh, const double* norm, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_finish_energy, dim3(1), dim3(64), 0, st, sums, nh, norm, out);
  return hipGetLastError();
}

hipError_t launch_gather_slots(const double* slot_val, const uint32_t* off, const uint32_t* idx,
                               const double* weight, int n_out, double* out, hipStream_t st) {
  if (n_out == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_slots, dim3((n_out + 255) / 256), dim3(256), 0, st, slot_val, off, idx, weight,
                     n_out, out);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, uint64_t n, double v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint64_t want = (n + 255) / 256;
  const int grid = int(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(k_fill_f64, dim3(grid), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_scale(int dtype, void* psi, uint64_t n_amp, const double* norm2, hipStream_t st) {
  const uint64_t want = (n_amp + 255) / 256;
  const int grid = int(want < 4096 ? want : 4096);
  if (dtype == 0)
    hipLaunchKernelGGL((k_scale<double2>), dim3(grid), dim3(256), 0, st, static_cast<double2*>(psi), n_amp, norm2);
  else
    hipLaunchKernelGGL((k_scale<float2>), dim3(grid), dim3(256), 0, st, static_cast<float2*>(psi), n_amp, norm2);
  return hipGetLastError();
}

hipError_t launch_gather_amps(int dtype, const void* psi, const uint64_t* idx, int64_t count, double* out,
                              hipStream_t st) {
  if (count == 0) return hipSuccess;
  const int grid = int((count + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL((k_gather_amps<double2>), dim3(grid), dim3(256), 0, st,
                       static_cast<const double2*>(psi), idx, count, out);
  else
    hipLaunchKernelGGL((k_gather_amps<float2>), dim3(grid), dim3(256), 0, st, static_cast<const float2*>(psi),
                       idx, count, out);
  return hipGetLastError();
}

}  // namespace q2sv
