// Rotation sweeps (Section 5.1, Eq. 11) and the reverse sweep of
// Algorithm 1 on gfx950: HF preparation, one fused run over the whole state,
// and LDS-tiled passes that apply many runs per HBM read and write of the
// state.  Tile passes are software-pipelined: while a block works on one
// tile-block in LDS, the loads of its next tile-block are already in flight
// into registers.
#include "device_common.h"
#include "launch.h"

namespace q2sv {

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
// One run over the whole state.  GRAD: 0 none (forward), 1 per-run parameter
// gradient, 2 per-string gradient.  Partials: partials[slot * nb + block].
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
        const uint64_t m2 = insert_zeros(t, run.sup_pack, run.n_sup) | rec.bits;
        const uint64_t m = m2 ^ run.x_loc;
        const unsigned sg = parity64(m2 & run.z0_loc);
        T a = psi[m], b = psi[m2];
        if (GRAD) {
          T la = lam[m], lb = lam[m2];
          wsum += grad_w(a, b, la, lb, sg, run.omega0);
          rot_pair(la, lb, c, s, sg, run.omega0);
          lam[m] = la;
          lam[m2] = lb;
        }
        rot_pair(a, b, c, s, sg, run.omega0);
        psi[m] = a;
        psi[m2] = b;
      }
      if (GRAD == 1) acc[0] += rec.a * wsum;
      if (GRAD == 2) {
#pragma unroll
        for (int k = 0; k < kMaxRunStrings; ++k) acc[k] += ((rec.eps_neg >> k) & 1u) ? -wsum : wsum;
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
        T la = lam[m], lb = lam[m2];
        const double w = grad_w(a, b, la, lb, sg, run.omega0);
        if (GRAD == 1) acc[0] += rec.a * w;
        if (GRAD == 2) {
#pragma unroll
          for (int k = 0; k < kMaxRunStrings; ++k) {
            const unsigned e = ((run.str_neg >> k) & 1u) ^ (__popc(p & pack_at(run.dpat_pack, k)) & 1u);
            acc[k] += e ? -w : w;
          }
        }
        rot_pair(la, lb, c, s, sg, run.omega0);
        lam[m] = la;
        lam[m2] = lb;
      }
      rot_pair(a, b, c, s, sg, run.omega0);
      psi[m] = a;
      psi[m2] = b;
    }
  } else {  // kRunDiag: psi[m] <- (c - i s (-1)^{|m & z0|}) psi[m]
    const uint64_t n_amp = uint64_t(1) << n;
    for (uint64_t m = tid0; m < n_amp; m += stride) {
      const unsigned sg = parity64(m & run.z0_loc);
      const unsigned p = run_pattern(run, m, 0);
      const RunRec rec = recs[run.rec_off + p];
      const R c = R(rec.c);
      const R s = (REV ? R(-rec.s) : R(rec.s)) * (sg ? R(-1) : R(1));
      const T a = psi[m];
      if (GRAD) {
        const T la = lam[m];
        double w = (double)la.x * (double)a.y - (double)la.y * (double)a.x;  // Im(conj(la) a)
        if (sg) w = -w;
        if (GRAD == 1) acc[0] += rec.a * w;
        if (GRAD == 2) {
#pragma unroll
          for (int k = 0; k < kMaxRunStrings; ++k) {
            const unsigned e = ((run.str_neg >> k) & 1u) ^ (__popc(p & pack_at(run.dpat_pack, k)) & 1u);
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
// In-LDS application of one run to a tile (forward) or to a psi/lam tile pair
// (reverse, with the gradient factor accumulated per lane).
// ---------------------------------------------------------------------------
template <typename T, int NT, bool REV, int GRAD>
__device__ __forceinline__ void tile_run(const RunDesc& run, const RunRec* __restrict__ recs, T* tp, T* tl,
                                         uint32_t nloc, uint64_t base, double (&acc)[GRAD == 2 ? kMaxRunStrings : 1]) {
  using R = typename Real<T>::type;
  const unsigned so = parity64(base & run.z0_out);
  const uint32_t xl = uint32_t(run.x_loc), zl = uint32_t(run.z0_loc);
  if (run.mode == kRunEnum) {
    const uint32_t np = nloc >> run.n_sup;
    for (int r = 0; r < run.n_rec; ++r) {
      const RunRec rec = recs[run.rec_off + r];
      const R c = R(rec.c), s = REV ? R(-rec.s) : R(rec.s);
      const uint32_t bits = uint32_t(rec.bits);
      double wsum = 0.0;
      for (uint32_t t = threadIdx.x; t < np; t += NT) {
        const uint32_t l2 = insert_zeros32(t, run.sup_pack, run.n_sup) | bits;
        const uint32_t l = l2 ^ xl;
        const unsigned sg = so ^ parity32(l2 & zl);
        T a = tp[l], b = tp[l2];
        if (REV) {
          T la = tl[l], lb = tl[l2];
          if (GRAD) wsum += grad_w(a, b, la, lb, sg, run.omega0);
          rot_pair(la, lb, c, s, sg, run.omega0);
          tl[l] = la;
          tl[l2] = lb;
        }
        rot_pair(a, b, c, s, sg, run.omega0);
        tp[l] = a;
        tp[l2] = b;
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
      const uint32_t l = insert_zero32(t, run.pivot);
      const uint32_t l2 = l ^ xl;
      const unsigned sg = so ^ parity32(l2 & zl);
      const unsigned p = run_pattern(run, l2, base);
      const RunRec rec = recs[run.rec_off + p];
      const R c = R(rec.c), s = REV ? R(-rec.s) : R(rec.s);
      T a = tp[l], b = tp[l2];
      if (REV) {
        T la = tl[l], lb = tl[l2];
        if (GRAD) {
          const double w = grad_w(a, b, la, lb, sg, run.omega0);
          if (GRAD == 1) acc[0] += rec.a * w;
          if (GRAD == 2) {
#pragma unroll
            for (int k = 0; k < kMaxRunStrings; ++k) {
              const unsigned e = ((run.str_neg >> k) & 1u) ^ (__popc(p & pack_at(run.dpat_pack, k)) & 1u);
              acc[k] += e ? -w : w;
            }
          }
        }
        rot_pair(la, lb, c, s, sg, run.omega0);
        tl[l] = la;
        tl[l2] = lb;
      }
      rot_pair(a, b, c, s, sg, run.omega0);
      tp[l] = a;
      tp[l2] = b;
    }
  } else {
    for (uint32_t l = threadIdx.x; l < nloc; l += NT) {
      const unsigned sg = so ^ parity32(l & zl);
      const unsigned p = run_pattern(run, l, base);
      const RunRec rec = recs[run.rec_off + p];
      const R c = R(rec.c), s = (REV ? R(-rec.s) : R(rec.s)) * (sg ? R(-1) : R(1));
      const T a = tp[l];
      if (REV) {
        const T la = tl[l];
        if (GRAD) {
          double w = (double)la.x * (double)a.y - (double)la.y * (double)a.x;
          if (sg) w = -w;
          if (GRAD == 1) acc[0] += rec.a * w;
          if (GRAD == 2) {
#pragma unroll
            for (int k = 0; k < kMaxRunStrings; ++k) {
              const unsigned e = ((run.str_neg >> k) & 1u) ^ (__popc(p & pack_at(run.dpat_pack, k)) & 1u);
              acc[k] += e ? -w : w;
            }
          }
        }
        tl[l] = cmake<T>(c * la.x + s * la.y, c * la.y - s * la.x);
      }
      tp[l] = cmake<T>(c * a.x + s * a.y, c * a.y - s * a.x);
    }
  }
}

// ---------------------------------------------------------------------------
// LDS tile, forward: load, apply every run of the pass, store.
// ---------------------------------------------------------------------------
// Copy the pass's run descriptors and records into LDS (once per block).
template <int NT>
__device__ __forceinline__ void stage_pass(const RunDesc* __restrict__ runs, int n_runs,
                                           const RunRec* __restrict__ recs, int n_recs, RunDesc* s_runs,
                                           RunRec* s_recs) {
  const uint4* src = reinterpret_cast<const uint4*>(runs);
  uint4* dst = reinterpret_cast<uint4*>(s_runs);
  const int w1 = n_runs * int(sizeof(RunDesc) / 16);
  for (int i = threadIdx.x; i < w1; i += NT) dst[i] = src[i];
  src = reinterpret_cast<const uint4*>(recs);
  dst = reinterpret_cast<uint4*>(s_recs);
  const int w2 = n_recs * int(sizeof(RunRec) / 16);
  for (int i = threadIdx.x; i < w2; i += NT) dst[i] = src[i];
}

template <typename T, int B, int NT>
__global__ void __launch_bounds__(NT) k_tile_forward(T* __restrict__ psi, FrameDesc fr,
                                                     const RunDesc* __restrict__ runs_g, int n_runs,
                                                     const RunRec* __restrict__ recs_g, int n_recs, uint64_t n_tb) {
  constexpr int PER = (1 << B) / NT;
  __shared__ T tile[1 << B];
  __shared__ FrameLut lut;
  __shared__ RunDesc runs[kMaxPassRuns];
  __shared__ RunRec recs[kMaxPassRecs];
  frame_lut_init<NT>(fr, lut);
  stage_pass<NT>(runs_g, n_runs, recs_g, n_recs, runs, recs);
  __syncthreads();
  const uint32_t nloc = 1u << fr.b;
  double dummy[1];
  Stage<T, PER> reg;
  uint64_t tb = blockIdx.x;
  if (tb < n_tb) tile_fetch<T, PER, NT>(psi, lut, frame_base(fr, tb), nloc, reg);
  for (; tb < n_tb; tb += gridDim.x) {
    const uint64_t base = frame_base(fr, tb);
    tile_put<T, PER, NT>(tile, nloc, reg);
    __syncthreads();
    const uint64_t nx = tb + gridDim.x;
    if (nx < n_tb) tile_fetch<T, PER, NT>(psi, lut, frame_base(fr, nx), nloc, reg);
    for (int ri = 0; ri < n_runs; ++ri) {
      tile_run<T, NT, false, 0>(runs[ri], recs, tile, nullptr, nloc, base, dummy);
      __syncthreads();
    }
    tile_store<T, PER, NT>(psi, lut, base, nloc, tile);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// LDS tile, reverse: psi and lam tiles; runs of the pass in pass order (the
// reverse of list order) each give their gradient factor, then are undone on
// both.  Gradient partials per local slot are summed per wavefront in LDS
// and written once per block: partials[slot_map[i] * nb + block].
// ---------------------------------------------------------------------------
template <int NW, int MAXS>
struct GradAcc {
  double v[MAXS][NW];
};

template <typename T, int B, int NT, int GRAD, int MAXS>
__global__ void __launch_bounds__(NT) k_tile_reverse(T* __restrict__ psi, T* __restrict__ lam, FrameDesc fr,
                                                     const RunDesc* __restrict__ runs_g, int n_runs,
                                                     const RunRec* __restrict__ recs_g, int n_recs,
                                                     const uint32_t* __restrict__ slot_map, int n_slots,
                                                     double* __restrict__ partials, uint32_t nb_stride,
                                                     uint64_t n_tb) {
  constexpr int NW = NT / 64;
  constexpr int PER = (1 << B) / NT;
  __shared__ T tp[1 << B];
  __shared__ T tl[1 << B];
  __shared__ FrameLut lut;
  __shared__ GradAcc<NW, MAXS> gacc;
  __shared__ RunDesc runs[kMaxPassRuns];
  __shared__ RunRec recs[kMaxPassRecs];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  frame_lut_init<NT>(fr, lut);
  stage_pass<NT>(runs_g, n_runs, recs_g, n_recs, runs, recs);
  for (int i = threadIdx.x; i < MAXS * NW; i += NT) (&gacc.v[0][0])[i] = 0.0;
  __syncthreads();
  const uint32_t nloc = 1u << fr.b;
  Stage<T, PER> rp, rl;
  uint64_t tb = blockIdx.x;
  if (tb < n_tb) {
    const uint64_t b0 = frame_base(fr, tb);
    tile_fetch<T, PER, NT>(psi, lut, b0, nloc, rp);
    tile_fetch<T, PER, NT>(lam, lut, b0, nloc, rl);
  }
  for (; tb < n_tb; tb += gridDim.x) {
    const uint64_t base = frame_base(fr, tb);
    tile_put<T, PER, NT>(tp, nloc, rp);
    tile_put<T, PER, NT>(tl, nloc, rl);
    __syncthreads();
    const uint64_t nx = tb + gridDim.x;
    if (nx < n_tb) {
      const uint64_t b1 = frame_base(fr, nx);
      tile_fetch<T, PER, NT>(psi, lut, b1, nloc, rp);
      tile_fetch<T, PER, NT>(lam, lut, b1, nloc, rl);
    }
    for (int ri = 0; ri < n_runs; ++ri) {
      const RunDesc run = runs[ri];
      double acc[GRAD == 2 ? kMaxRunStrings : 1];
#pragma unroll
      for (int k = 0; k < (GRAD == 2 ? kMaxRunStrings : 1); ++k) acc[k] = 0.0;
      tile_run<T, NT, true, GRAD>(run, recs, tp, tl, nloc, base, acc);
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
    tile_store<T, PER, NT>(psi, lut, base, nloc, tp);
    tile_store<T, PER, NT>(lam, lut, base, nloc, tl);
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
// launchers
// ---------------------------------------------------------------------------
template <typename T>
static hipError_t run_full_t(bool rev, int grad, void* psi, void* lam, const RunDesc& run, const RunRec* recs,
                             double* partials, int n, uint32_t nb, int grid, hipStream_t st) {
  T* p = static_cast<T*>(psi);
  T* l = static_cast<T*>(lam);
  if (!rev)
    hipLaunchKernelGGL((k_run_full<T, false, 0>), dim3(grid), dim3(256), 0, st, p, l, run, recs, partials, n, nb);
  else if (grad == 0)
    hipLaunchKernelGGL((k_run_full<T, true, 0>), dim3(grid), dim3(256), 0, st, p, l, run, recs, partials, n, nb);
  else if (grad == 1)
    hipLaunchKernelGGL((k_run_full<T, true, 1>), dim3(grid), dim3(256), 0, st, p, l, run, recs, partials, n, nb);
  else
    hipLaunchKernelGGL((k_run_full<T, true, 2>), dim3(grid), dim3(256), 0, st, p, l, run, recs, partials, n, nb);
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
                               const RunRec* recs, int n_recs, uint64_t n_tb, int grid, hipStream_t st) {
  if (n_runs > kMaxPassRuns || n_recs > kMaxPassRecs) return hipErrorInvalidValue;
  if (dtype == 0)
    hipLaunchKernelGGL((k_tile_forward<double2, kTileFwdC128, kTileThreads>), dim3(grid), dim3(kTileThreads), 0,
                       st, static_cast<double2*>(psi), fr, runs, n_runs, recs, n_recs, n_tb);
  else
    hipLaunchKernelGGL((k_tile_forward<float2, kTileFwdC64, kTileThreads>), dim3(grid), dim3(kTileThreads), 0,
                       st, static_cast<float2*>(psi), fr, runs, n_runs, recs, n_recs, n_tb);
  return hipGetLastError();
}

template <typename T, int B>
static hipError_t tile_reverse_t(int grad, void* psi, void* lam, const FrameDesc& fr, const RunDesc* runs,
                                 int n_runs, const RunRec* recs, int n_recs, const uint32_t* slot_map, int n_slots,
                                 double* partials, uint32_t nb, uint64_t n_tb, int grid, hipStream_t st) {
  T* p = static_cast<T*>(psi);
  T* l = static_cast<T*>(lam);
  if (grad == 0)
    hipLaunchKernelGGL((k_tile_reverse<T, B, kTileThreads, 0, 1>), dim3(grid), dim3(kTileThreads), 0, st, p, l,
                       fr, runs, n_runs, recs, n_recs, slot_map, n_slots, partials, nb, n_tb);
  else if (grad == 1)
    hipLaunchKernelGGL((k_tile_reverse<T, B, kTileThreads, 1, kMaxPassSlots>), dim3(grid), dim3(kTileThreads), 0,
                       st, p, l, fr, runs, n_runs, recs, n_recs, slot_map, n_slots, partials, nb, n_tb);
  else
    hipLaunchKernelGGL((k_tile_reverse<T, B, kTileThreads, 2, kMaxPassSlots>), dim3(grid), dim3(kTileThreads), 0,
                       st, p, l, fr, runs, n_runs, recs, n_recs, slot_map, n_slots, partials, nb, n_tb);
  return hipGetLastError();
}

hipError_t launch_tile_reverse(int dtype, int grad, void* psi, void* lam, const FrameDesc& fr,
                               const RunDesc* runs, int n_runs, const RunRec* recs, int n_recs,
                               const uint32_t* slot_map, int n_slots, double* partials, uint32_t nb_stride,
                               uint64_t n_tb, int grid, hipStream_t st) {
  if (n_runs > kMaxPassRuns || n_recs > kMaxPassRecs || n_slots > kMaxPassSlots) return hipErrorInvalidValue;
  if (dtype == 0)
    return tile_reverse_t<double2, kTileTwoC128>(grad, psi, lam, fr, runs, n_runs, recs, n_recs, slot_map,
                                                 n_slots, partials, nb_stride, n_tb, grid, st);
  return tile_reverse_t<float2, kTileTwoC64>(grad, psi, lam, fr, runs, n_runs, recs, n_recs, slot_map, n_slots,
                                             partials, nb_stride, n_tb, grid, st);
}

}  // namespace q2sv
