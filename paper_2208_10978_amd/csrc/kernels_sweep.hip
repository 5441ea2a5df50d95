// Rotation sweeps (Section 5.1, Eq. 11) and the reverse sweep of
// Algorithm 1 on gfx950: HF preparation, one fused run over the whole state,
// and LDS-tiled passes that apply many runs per HBM read and write of the
// state.  Tile passes are software-pipelined: while a block works on one
// tile-block in LDS, the loads of its next tile-block are already in flight
// into registers.  Inside a tile, runs are grouped in segments whose pairs
// stay within per-wavefront regions, so the block synchronises once per
// segment instead of once per run.
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
// In-LDS application of one run to this wavefront's region of a tile
// (forward), or of a psi/lam tile pair (reverse, with the gradient factor
// accumulated per lane).  Walk position t = lane + 64 j: the lane's bits are
// deposited once per run with one and-or per bit from per-lane masks, the
// bits of j (uniform) on the scalar unit; LDS slots follow by linearity.
// ---------------------------------------------------------------------------
struct LaneBits {
  uint32_t m[kWalkLaneBits];  // all ones where the lane index has bit i
  __device__ explicit LaneBits(uint32_t lane) {
#pragma unroll
    for (int i = 0; i < kWalkLaneBits; ++i) m[i] = 0u - ((lane >> i) & 1u);
  }
};

// the lane's part of the walk index and of its LDS slot
__device__ __forceinline__ void lane_walk(const RunDesc& run, const LaneBits& lb, uint32_t& dl, uint32_t& ds) {
  dl = 0;
  ds = 0;
#pragma unroll
  for (int i = 0; i < kWalkLaneBits; ++i) {
    dl |= lb.m[i] & run.dep_p[i];
    ds ^= lb.m[i] & run.dep_q[i];
  }
}

template <unsigned OM, typename V>
__device__ __forceinline__ void rot_pair_om(V& a, V& b, typename Real<V>::type c, typename Real<V>::type s,
                                            unsigned sgn) {
  rot_pair(a, b, c, s, sgn, OM);
}

template <unsigned OM, typename V>
__device__ __forceinline__ double grad_w_om(V pa, V pb, V la, V lb, unsigned sgn) {
  return grad_w(pa, pb, la, lb, sgn, OM);
}

// kRunEnum: every record's pairs, with the phase power omega0 = OM fixed
template <typename T, bool REV, int GRAD, unsigned OM>
__device__ __forceinline__ void enum_walk(const RunDesc& run, const RunRec* __restrict__ recs, T* tp, T* tl,
                                          uint32_t dl, uint32_t ds, unsigned zlane_par, bool lane_on, unsigned so,
                                          uint32_t wbits, double (&acc)[GRAD == 2 ? kMaxRunStrings : 1]) {
  using R = typename Real<T>::type;
  const uint32_t xl = uint32_t(run.x_loc), zl = uint32_t(run.z0_loc);
  const uint32_t sx = lds_swz(xl);  // slot(l ^ x) = slot(l) ^ slot(x)
  const uint32_t nj = run.walk_log > kWalkLaneBits ? 1u << (run.walk_log - kWalkLaneBits) : 1u;
  if (nj == 1u) {
    // one position per lane: the pairs of different records are disjoint, so
    // the reads of RB records leave together, then their updates and writes
    // (one LDS round trip per RB records instead of one per record)
    constexpr int RB = 2;
    for (uint32_t r0 = 0; r0 < run.n_rec; r0 += RB) {
      R c[RB], s[RB];
      uint32_t s1[RB], s2[RB];
      unsigned sg[RB];
      T a[RB], b[RB], la[RB], lb[RB];
      double w[RB];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        w[q] = 0.0;
        if (r0 + uint32_t(q) < run.n_rec) {
          const RunRec rec = recs[run.rec_off + r0 + uint32_t(q)];
          c[q] = R(rec.c);
          s[q] = REV ? R(-rec.s) : R(rec.s);
          const uint32_t rest = uint32_t(rec.bits) | wbits;  // uniform
          sg[q] = zlane_par ^ so ^ parity32(rest & zl);
          s2[q] = ds ^ lds_swz(rest);  // slot of m'
          s1[q] = s2[q] ^ sx;          // slot of m
          if (lane_on) {
            a[q] = tp[s1[q]];
            b[q] = tp[s2[q]];
            if (REV) {
              la[q] = tl[s1[q]];
              lb[q] = tl[s2[q]];
            }
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        if (r0 + uint32_t(q) < run.n_rec && lane_on) {
          if (REV) {
            if (GRAD) w[q] = grad_w_om<OM>(a[q], b[q], la[q], lb[q], sg[q]);
            rot_pair_om<OM>(la[q], lb[q], c[q], s[q], sg[q]);
            tl[s1[q]] = la[q];
            tl[s2[q]] = lb[q];
          }
          rot_pair_om<OM>(a[q], b[q], c[q], s[q], sg[q]);
          tp[s1[q]] = a[q];
          tp[s2[q]] = b[q];
        }
      }
      if (GRAD) {
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          if (r0 + uint32_t(q) >= run.n_rec) break;
          const RunRec& rec = recs[run.rec_off + r0 + uint32_t(q)];
          if (GRAD == 1) acc[0] += rec.a * w[q];
          if (GRAD == 2) {
#pragma unroll
            for (int k = 0; k < kMaxRunStrings; ++k) acc[k] += ((rec.eps_neg >> k) & 1u) ? -w[q] : w[q];
          }
        }
      }
    }
    (void)dl;
    return;
  }
  for (uint32_t r = 0; r < run.n_rec; ++r) {
    const RunRec rec = recs[run.rec_off + r];
    const R c = R(rec.c), s = REV ? R(-rec.s) : R(rec.s);
    double wsum = 0.0;
    for (uint32_t j = 0; j < nj; ++j) {
      const uint32_t rest = deposit_bits(j, run.hi_mask) | uint32_t(rec.bits) | wbits;  // uniform
      const uint32_t srest = lds_swz(rest);
      const unsigned prest = so ^ parity32(rest & zl);
      if (lane_on) {
        const uint32_t s2 = ds ^ srest, s1 = s2 ^ sx;  // slots of m' and m
        const unsigned sg = zlane_par ^ prest;
        T a = tp[s1], b = tp[s2];
        if (REV) {
          T la = tl[s1], lb = tl[s2];
          if (GRAD) wsum += grad_w_om<OM>(a, b, la, lb, sg);
          rot_pair_om<OM>(la, lb, c, s, sg);
          tl[s1] = la;
          tl[s2] = lb;
        }
        rot_pair_om<OM>(a, b, c, s, sg);
        tp[s1] = a;
        tp[s2] = b;
      }
    }
    (void)dl;
    if (GRAD == 1) acc[0] += rec.a * wsum;
    if (GRAD == 2) {
#pragma unroll
      for (int k = 0; k < kMaxRunStrings; ++k) acc[k] += ((rec.eps_neg >> k) & 1u) ? -wsum : wsum;
    }
  }
}

// Short runs (kRunEnum, at most two records, one position per lane): every
// uniform quantity comes precomputed with the descriptor head, and the slot
// and sign of a pair follow from the lane part and per-record constants.
//
// The head is read in one batch and held in SGPRs before the first branch of
// the run: a field first used under a branch would otherwise be loaded there,
// and every branch level would wait for its own scalar-cache round trip.
struct ShortHead {
  uint32_t short_form, n_rec, omega0, walk_log, zlane, sx, slot;
  uint32_t z0_loc;
  uint64_t z0_out;
  uint32_t dep_q[kWalkLaneBits];
  uint32_t sb[2], pb[2];
  double c[2], s[2], a[2];
};

template <int GRAD>
__device__ __forceinline__ ShortHead load_head(const RunDesc& run) {
  ShortHead h;
  h.short_form = run.short_form;
  h.n_rec = run.n_rec;
  h.omega0 = run.omega0;
  h.walk_log = run.walk_log;
  h.zlane = run.zlane;
  h.sx = run.sx;
  h.slot = run.slot;
  h.z0_loc = uint32_t(run.z0_loc);
  h.z0_out = run.z0_out;
#pragma unroll
  for (int i = 0; i < kWalkLaneBits; ++i) h.dep_q[i] = run.dep_q[i];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    h.sb[r] = run.rec_sbits[r];
    h.pb[r] = run.rec_pbits[r];
    h.c[r] = run.rec_c[r];
    h.s[r] = run.rec_s[r];
    h.a[r] = GRAD == 1 ? run.rec_a[r] : 0.0;
  }
  sgpr_here(h.short_form);
  sgpr_here(h.n_rec);
  sgpr_here(h.omega0);
  sgpr_here(h.walk_log);
  sgpr_here(h.zlane);
  sgpr_here(h.sx);
  sgpr_here(h.slot);
  sgpr_here(h.z0_loc);
  sgpr_here(h.z0_out);
#pragma unroll
  for (int i = 0; i < kWalkLaneBits; ++i) sgpr_here(h.dep_q[i]);
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    sgpr_here(h.sb[r]);
    sgpr_here(h.pb[r]);
    sgpr_here(h.c[r]);
    sgpr_here(h.s[r]);
    if (GRAD == 1) sgpr_here(h.a[r]);
  }
  return h;
}

// One record, or two (every double excitation): the records' pairs are
// disjoint, so all LDS reads of the run leave first, then the updates, then
// the writes; one LDS round trip per run.
// REALV (reverse sweep, real rotation, psi and lam real): only the real
// parts are read, updated and written; the imaginary parts stay zero.
template <typename T, bool REV, int GRAD, unsigned OM, int NR, bool REALV = false>
__device__ __forceinline__ void short_walk(const ShortHead& h, const RunDesc& run, T* tp, T* tl, uint32_t ds,
                                           unsigned sgn0, uint32_t swb, bool lane_on,
                                           double (&acc)[GRAD == 2 ? kMaxRunStrings : 1]) {
  using R = typename Real<T>::type;
  static_assert(!REALV || (REV && (OM & 1u)), "the real walk is for real rotations in the reverse sweep");
  double w[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) w[r] = 0.0;
  if (lane_on) {
    uint32_t s1[NR], s2[NR];
    T a[NR], b[NR], la[NR], lb[NR];
    R ar[NR], br[NR], lar[NR], lbr[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      s2[r] = ds ^ h.sb[r] ^ swb;  // slot of m'
      s1[r] = s2[r] ^ h.sx;        // slot of m
      if (REALV) {
        ar[r] = tp[s1[r]].x;
        br[r] = tp[s2[r]].x;
        lar[r] = tl[s1[r]].x;
        lbr[r] = tl[s2[r]].x;
      } else {
        a[r] = tp[s1[r]];
        b[r] = tp[s2[r]];
        if (REV) {
          la[r] = tl[s1[r]];
          lb[r] = tl[s2[r]];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const R c = R(h.c[r]), s = REV ? R(-h.s[r]) : R(h.s[r]);
      const unsigned sg = sgn0 ^ h.pb[r];
      if (REALV) {
        if (GRAD) w[r] = grad_w_real<OM>(ar[r], br[r], lar[r], lbr[r], sg);
        rot_pair_real<OM>(lar[r], lbr[r], c, s, sg);
        rot_pair_real<OM>(ar[r], br[r], c, s, sg);
        continue;
      }
      if (REV) {
        if (GRAD) w[r] = grad_w_om<OM>(a[r], b[r], la[r], lb[r], sg);
        rot_pair_om<OM>(la[r], lb[r], c, s, sg);
      }
      rot_pair_om<OM>(a[r], b[r], c, s, sg);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (REALV) {
        tp[s1[r]].x = ar[r];
        tp[s2[r]].x = br[r];
        tl[s1[r]].x = lar[r];
        tl[s2[r]].x = lbr[r];
        continue;
      }
      tp[s1[r]] = a[r];
      tp[s2[r]] = b[r];
      if (REV) {
        tl[s1[r]] = la[r];
        tl[s2[r]] = lb[r];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (GRAD == 1) acc[0] += h.a[r] * w[r];
    if (GRAD == 2) {
#pragma unroll
      for (int k = 0; k < kMaxRunStrings; ++k) acc[k] += ((run.rec_eps[r] >> k) & 1u) ? -w[r] : w[r];
    }
  }
}

// Two records whose walks fit half a wavefront (walk_log < 6, every double
// excitation in an 8-region tile), reverse sweep: lane bit walk_log picks the
// record, so each lane updates one pair of psi and one of lambda and no lane
// idles (the forward sweep, with half the work per pair, gains nothing).  The record's constants are
// selected per lane; the lane bits below walk_log are the walk position.
template <typename T, bool REV, int GRAD, unsigned OM, bool REALV = false>
__device__ __forceinline__ void short_walk_split(const ShortHead& h, const RunDesc& run, T* tp, T* tl, uint32_t ds,
                                                 unsigned sgn0, uint32_t swb, uint32_t lane,
                                                 double (&acc)[GRAD == 2 ? kMaxRunStrings : 1]) {
  using R = typename Real<T>::type;
  static_assert(!REALV || (REV && (OM & 1u)), "the real walk is for real rotations in the reverse sweep");
  const bool r1 = (lane >> h.walk_log) & 1u;
  const bool lane_on = lane < (2u << h.walk_log);
  double w = 0.0;
  if (lane_on && REALV) {
    const uint32_t s2 = ds ^ (r1 ? h.sb[1] : h.sb[0]) ^ swb;  // slot of m'
    const uint32_t s1 = s2 ^ h.sx;                            // slot of m
    R a = tp[s1].x, b = tp[s2].x, la = tl[s1].x, lb = tl[s2].x;
    const R c = R(r1 ? h.c[1] : h.c[0]);
    const R s = R(-(r1 ? h.s[1] : h.s[0]));
    const unsigned sg = sgn0 ^ (r1 ? h.pb[1] : h.pb[0]);
    if (GRAD) w = grad_w_real<OM>(a, b, la, lb, sg);
    rot_pair_real<OM>(la, lb, c, s, sg);
    rot_pair_real<OM>(a, b, c, s, sg);
    tl[s1].x = la;
    tl[s2].x = lb;
    tp[s1].x = a;
    tp[s2].x = b;
  } else if (lane_on) {
    const uint32_t s2 = ds ^ (r1 ? h.sb[1] : h.sb[0]) ^ swb;  // slot of m'
    const uint32_t s1 = s2 ^ h.sx;                            // slot of m
    T a = tp[s1], b = tp[s2];
    T la, lb;
    if (REV) {
      la = tl[s1];
      lb = tl[s2];
    }
    const R c = R(r1 ? h.c[1] : h.c[0]);
    const R s = REV ? R(-(r1 ? h.s[1] : h.s[0])) : R(r1 ? h.s[1] : h.s[0]);
    const unsigned sg = sgn0 ^ (r1 ? h.pb[1] : h.pb[0]);
    if (REV) {
      if (GRAD) w = grad_w_om<OM>(a, b, la, lb, sg);
      rot_pair_om<OM>(la, lb, c, s, sg);
      tl[s1] = la;
      tl[s2] = lb;
    }
    rot_pair_om<OM>(a, b, c, s, sg);
    tp[s1] = a;
    tp[s2] = b;
  }
  if (GRAD == 1) acc[0] += (r1 ? h.a[1] : h.a[0]) * w;
  if (GRAD == 2) {
    const uint32_t eps = r1 ? run.rec_eps[1] : run.rec_eps[0];
#pragma unroll
    for (int k = 0; k < kMaxRunStrings; ++k) acc[k] += ((eps >> k) & 1u) ? -w : w;
  }
}

// real: psi and lam are real (reverse sweep of a list of real rotations), so
// a run with omega0 = 1 or 3 takes the real walk
template <typename T, bool REV, int GRAD>
__device__ __forceinline__ void short_run(const ShortHead& h, const RunDesc& run, T* tp, T* tl, uint64_t base,
                                          uint32_t wbits, uint32_t swb, uint32_t lane, const LaneBits& lb,
                                          double (&acc)[GRAD == 2 ? kMaxRunStrings : 1], bool real = false) {
  uint32_t ds = 0;
#pragma unroll
  for (int i = 0; i < kWalkLaneBits; ++i) ds ^= lb.m[i] & h.dep_q[i];
  const unsigned sgn0 = (parity64(base & h.z0_out) ^ parity32(wbits & h.z0_loc)) ^ parity32(lane & h.zlane);
  const bool lane_on = lane < (1u << h.walk_log);
  const bool split = REV && h.n_rec == 2 && h.walk_log < uint32_t(kWalkLaneBits);
#define Q2SV_SHORT(OMV, RV)                                                                          \
  {                                                                                                  \
    if (split) short_walk_split<T, REV, GRAD, OMV, RV>(h, run, tp, tl, ds, sgn0, swb, lane, acc);        \
    else if (h.n_rec == 2) short_walk<T, REV, GRAD, OMV, 2, RV>(h, run, tp, tl, ds, sgn0, swb, lane_on, acc); \
    else short_walk<T, REV, GRAD, OMV, 1, RV>(h, run, tp, tl, ds, sgn0, swb, lane_on, acc);                \
  }
  switch (h.omega0 & 3u) {
    case 0: Q2SV_SHORT(0, false) break;
    case 1:
      if constexpr (REV) {
        if (real) Q2SV_SHORT(1, true) else Q2SV_SHORT(1, false)
      } else {
        Q2SV_SHORT(1, false)
      }
      break;
    case 2: Q2SV_SHORT(2, false) break;
    default:
      if constexpr (REV) {
        if (real) Q2SV_SHORT(3, true) else Q2SV_SHORT(3, false)
      } else {
        Q2SV_SHORT(3, false)
      }
      break;
  }
#undef Q2SV_SHORT
}

template <typename T, bool REV, int GRAD>
__device__ __forceinline__ void tile_run(const RunDesc& run, const RunRec* __restrict__ recs, T* tp, T* tl,
                                         uint64_t base, uint32_t wbits, uint32_t lane, const LaneBits& lbits,
                                         double (&acc)[GRAD == 2 ? kMaxRunStrings : 1]) {
  using R = typename Real<T>::type;
  const unsigned so = parity64(base & run.z0_out);
  const uint32_t xl = uint32_t(run.x_loc), zl = uint32_t(run.z0_loc);
  const uint32_t sx = lds_swz(xl);
  uint32_t dl, ds;
  lane_walk(run, lbits, dl, ds);
  const bool lane_on = run.walk_log >= kWalkLaneBits || lane < (1u << run.walk_log);
  const uint32_t nj = run.walk_log > kWalkLaneBits ? 1u << (run.walk_log - kWalkLaneBits) : 1u;
  if (run.mode == kRunEnum) {
    const unsigned zp = parity32(lane & run.zlane);
    switch (run.omega0 & 3u) {
      case 0: enum_walk<T, REV, GRAD, 0>(run, recs, tp, tl, dl, ds, zp, lane_on, so, wbits, acc); break;
      case 1: enum_walk<T, REV, GRAD, 1>(run, recs, tp, tl, dl, ds, zp, lane_on, so, wbits, acc); break;
      case 2: enum_walk<T, REV, GRAD, 2>(run, recs, tp, tl, dl, ds, zp, lane_on, so, wbits, acc); break;
      default: enum_walk<T, REV, GRAD, 3>(run, recs, tp, tl, dl, ds, zp, lane_on, so, wbits, acc); break;
    }
  } else if (run.mode == kRunFull) {
    for (uint32_t j = 0; j < nj; ++j) {
      const uint32_t rest = deposit_bits(j, run.hi_mask) | wbits;
      if (!lane_on) continue;
      const uint32_t l = dl | rest;  // pivot bit clear
      const uint32_t l2 = l ^ xl;
      const uint32_t s1 = ds ^ lds_swz(rest), s2 = s1 ^ sx;
      const unsigned sg = so ^ parity32(l2 & zl);
      const unsigned p = run_pattern(run, l2, base);
      const RunRec rec = recs[run.rec_off + p];
      const R c = R(rec.c), s = REV ? R(-rec.s) : R(rec.s);
      T a = tp[s1], b = tp[s2];
      if (REV) {
        T la = tl[s1], lb = tl[s2];
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
        tl[s1] = la;
        tl[s2] = lb;
      }
      rot_pair(a, b, c, s, sg, run.omega0);
      tp[s1] = a;
      tp[s2] = b;
    }
  } else {
    for (uint32_t j = 0; j < nj; ++j) {
      const uint32_t rest = deposit_bits(j, run.hi_mask) | wbits;
      if (!lane_on) continue;
      const uint32_t l = dl | rest;
      const uint32_t s1 = ds ^ lds_swz(rest);
      const unsigned sg = so ^ parity32(l & zl);
      const unsigned p = run_pattern(run, l, base);
      const RunRec rec = recs[run.rec_off + p];
      const R c = R(rec.c), s = (REV ? R(-rec.s) : R(rec.s)) * (sg ? R(-1) : R(1));
      const T a = tp[s1];
      if (REV) {
        const T la = tl[s1];
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
        tl[s1] = cmake<T>(c * la.x + s * la.y, c * la.y - s * la.x);
      }
      tp[s1] = cmake<T>(c * a.x + s * a.y, c * a.y - s * a.x);
    }
  }
}

// ---------------------------------------------------------------------------
// LDS tile, forward: load, apply every run of the pass, store.  Within a
// segment each wavefront runs through the segment's runs on its own region;
// a block barrier separates segments.  Descriptors are read in place through
// scalar loads.
//
// Full tiles (FULL): the next tile's loads leave before the runs of this one;
// after the runs each thread takes its own slots into registers, puts the
// next tile's amplitudes in their place and only then sends this tile's
// stores, so stores stay in flight over the next tile's runs and nothing
// waits for them.  Frames narrower than B (states of fewer than B qubits)
// take the guarded loop.
// ---------------------------------------------------------------------------
template <typename T, int B, int NT, bool FULL, int MINB>
__global__ void __launch_bounds__(NT, MINB) k_tile_forward(T* __restrict__ psi, FrameDesc fr,
                                                     const RunDesc* __restrict__ runs,
                                                     const RunRec* __restrict__ recs,
                                                     const SegDesc* __restrict__ segs, int n_segs, uint64_t n_tb) {
  constexpr int PER = (1 << B) / NT;
  __shared__ T tile[1 << B];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const LaneBits lbits(lane);
  double dummy[1];
  auto apply_runs = [&](uint64_t base) {
    for (int si = 0; si < n_segs; ++si) {
      const SegDesc sg = segs[si];
      if (wave < (1u << __popc(sg.wb_mask))) {
        const uint32_t wbits = region_bits_of(sg.wb_mask, wave), swb = lds_swz(wbits);
        for (uint32_t ri = sg.first; ri < sg.first + sg.count; ++ri) {
          const ShortHead h = load_head<0>(runs[ri]);
          if (h.short_form)
            short_run<T, false, 0>(h, runs[ri], tile, nullptr, base, wbits, swb, lane, lbits, dummy);
          else
            tile_run<T, false, 0>(runs[ri], recs, tile, nullptr, base, wbits, lane, lbits, dummy);
        }
      }
      __syncthreads();
    }
  };
  Stage<T, PER> reg;
  uint64_t tb = blockIdx.x;
  if constexpr (FULL) {
    const TileAddr<NT, PER> ta(fr);
    Stage<T, PER> out;
    if (tb < n_tb) {
      tile_fetch_full<T, PER, NT>(psi, ta, frame_base(fr, tb), reg);
      tile_put_full<T, PER, NT>(tile, reg);
    }
    __syncthreads();
    for (; tb < n_tb; tb += gridDim.x) {
      const uint64_t base = frame_base(fr, tb);
      const uint64_t nx = tb + gridDim.x;
      if (nx < n_tb) tile_fetch_full<T, PER, NT>(psi, ta, frame_base(fr, nx), reg);
      apply_runs(base);
      tile_take<T, PER, NT>(tile, out);
      if (nx < n_tb) tile_put_full<T, PER, NT>(tile, reg);
      tile_send<T, PER, NT>(psi, ta, base, out);
      __syncthreads();
    }
  } else {
    __shared__ FrameLut lut;
    frame_lut_init<NT>(fr, lut);
    __syncthreads();
    const uint32_t nloc = 1u << fr.b;
    if (tb < n_tb) tile_fetch<T, PER, NT>(psi, lut, frame_base(fr, tb), nloc, reg);
    for (; tb < n_tb; tb += gridDim.x) {
      const uint64_t base = frame_base(fr, tb);
      tile_put<T, PER, NT>(tile, nloc, reg);
      __syncthreads();
      const uint64_t nx = tb + gridDim.x;
      if (nx < n_tb) tile_fetch<T, PER, NT>(psi, lut, frame_base(fr, nx), nloc, reg);
      apply_runs(base);
      tile_store<T, PER, NT>(psi, lut, base, nloc, tile);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// LDS tile, reverse: psi and lam tiles; runs of the pass in pass order (the
// reverse of list order) each give their gradient factor, then are undone on
// both.  Gradient partials per local slot are summed per row of 16 lanes
// in LDS (one cell per wavefront and row) and written once per block in a
// fixed order: partials[slot_map[i] * nb + block].
// ---------------------------------------------------------------------------
template <int NW, int MAXS>
struct GradAcc {
  double v[MAXS][NW * 4];  // per slot: one cell per (wavefront, row of 16 lanes)
};

template <typename T, int B, int NT, int GRAD, int MAXS, bool FULL, int MINB>
__global__ void __launch_bounds__(NT, MINB) k_tile_reverse(T* __restrict__ psi, T* __restrict__ lam, FrameDesc fr,
                                                     const RunDesc* __restrict__ runs,
                                                     const RunRec* __restrict__ recs,
                                                     const SegDesc* __restrict__ segs, int n_segs,
                                                     const uint32_t* __restrict__ slot_map, int n_slots,
                                                     double* __restrict__ partials, uint32_t nb_stride,
                                                     uint64_t n_tb, const double* __restrict__ imag_count) {
  constexpr int NW = NT / 64;
  constexpr int PER = (1 << B) / NT;
  __shared__ T tp[1 << B];
  __shared__ T tl[1 << B];
  // imag_count (device, may be NULL): nonzero imaginary parts of psi and lam,
  // given for a list of real rotations only; zero lets real runs take the
  // real walk (psi and lam then stay real through the whole sweep)
  const bool real = imag_count && *imag_count == 0.0;
  __shared__ GradAcc<NW, MAXS> gacc;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const LaneBits lbits(lane);
  for (int i = threadIdx.x; i < MAXS * NW * 4; i += NT) (&gacc.v[0][0])[i] = 0.0;
  auto apply_runs = [&](uint64_t base) {
    for (int si = 0; si < n_segs; ++si) {
      const SegDesc sg = segs[si];
      if (wave < (1u << __popc(sg.wb_mask))) {
        const uint32_t wbits = region_bits_of(sg.wb_mask, wave), swb = lds_swz(wbits);
        for (uint32_t ri = sg.first; ri < sg.first + sg.count; ++ri) {
          const RunDesc& run = runs[ri];
          double acc[GRAD == 2 ? kMaxRunStrings : 1];
#pragma unroll
          for (int k = 0; k < (GRAD == 2 ? kMaxRunStrings : 1); ++k) acc[k] = 0.0;
          const ShortHead h = load_head<GRAD>(run);
          if (h.short_form) short_run<T, true, GRAD>(h, run, tp, tl, base, wbits, swb, lane, lbits, acc, real);
          else tile_run<T, true, GRAD>(run, recs, tp, tl, base, wbits, lane, lbits, acc);
          if (GRAD) {
            const int nk = GRAD == 2 ? int(run.n_str) : 1;
            for (int k = 0; k < (GRAD == 2 ? kMaxRunStrings : 1); ++k) {
              if (k >= nk) break;
              // row sums only: the row's last lane adds into the cell of its
              // (wavefront, row), which nothing else writes
              const double v = row_sum(acc[k]);
              if ((lane & 15u) == 15u) lds_add(&gacc.v[h.slot + k][wave * 4 + (lane >> 4)], v);
            }
          }
        }
      }
      __syncthreads();
    }
  };
  Stage<T, PER> rp, rl;
  uint64_t tb = blockIdx.x;
  if constexpr (FULL) {
    // as in the forward pass: next loads before the runs, stores after the
    // next tile is in place
    const TileAddr<NT, PER> ta(fr);
    Stage<T, PER> op, ol;
    if (tb < n_tb) {
      const uint64_t b0 = frame_base(fr, tb);
      tile_fetch_full<T, PER, NT>(psi, ta, b0, rp);
      tile_fetch_full<T, PER, NT>(lam, ta, b0, rl);
      tile_put_full<T, PER, NT>(tp, rp);
      tile_put_full<T, PER, NT>(tl, rl);
    }
    __syncthreads();
    for (; tb < n_tb; tb += gridDim.x) {
      const uint64_t base = frame_base(fr, tb);
      const uint64_t nx = tb + gridDim.x;
      if (nx < n_tb) {
        const uint64_t b1 = frame_base(fr, nx);
        tile_fetch_full<T, PER, NT>(psi, ta, b1, rp);
        tile_fetch_full<T, PER, NT>(lam, ta, b1, rl);
      }
      apply_runs(base);
      tile_take<T, PER, NT>(tp, op);
      tile_take<T, PER, NT>(tl, ol);
      if (nx < n_tb) {
        tile_put_full<T, PER, NT>(tp, rp);
        tile_put_full<T, PER, NT>(tl, rl);
      }
      tile_send<T, PER, NT>(psi, ta, base, op);
      tile_send<T, PER, NT>(lam, ta, base, ol);
      __syncthreads();
    }
  } else {
    __shared__ FrameLut lut;
    frame_lut_init<NT>(fr, lut);
    __syncthreads();
    const uint32_t nloc = 1u << fr.b;
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
      apply_runs(base);
      tile_store<T, PER, NT>(psi, lut, base, nloc, tp);
      tile_store<T, PER, NT>(lam, lut, base, nloc, tl);
      __syncthreads();
    }
  }
  if (GRAD) {
    __syncthreads();
    for (int i = threadIdx.x; i < n_slots; i += NT) {
      double s = 0.0;
      for (int w = 0; w < NW * 4; ++w) s += gacc.v[i][w];
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
  return by_dtype(dtype, [&](auto tag) {
    using T = decltype(tag);
    hipLaunchKernelGGL((k_fill_basis<T>), dim3(grid), dim3(256), 0, st, static_cast<T*>(psi), n_amp, k);
  });
}

hipError_t launch_run_full(int dtype, bool rev, int grad, void* psi, void* lam, const RunDesc& run,
                           const RunRec* recs, double* partials, int n, uint32_t nb_stride, int grid,
                           hipStream_t st) {
  if (dtype == 0) return run_full_t<double2>(rev, grad, psi, lam, run, recs, partials, n, nb_stride, grid, st);
  if (dtype == 1) return run_full_t<float2>(rev, grad, psi, lam, run, recs, partials, n, nb_stride, grid, st);
  return run_full_t<R64>(rev, grad, psi, lam, run, recs, partials, n, nb_stride, grid, st);
}

template <typename T, int B, int MINB = 1>
static hipError_t tile_forward_t(void* psi, const FrameDesc& fr, const RunDesc* runs, const RunRec* recs,
                                 const SegDesc* segs, int n_segs, uint64_t n_tb, int grid, hipStream_t st) {
  T* p = static_cast<T*>(psi);
  if (fr.b == B)
    hipLaunchKernelGGL((k_tile_forward<T, B, kTileThreads, true, MINB>), dim3(grid), dim3(kTileThreads), 0, st, p,
                       fr, runs, recs, segs, n_segs, n_tb);
  else
    hipLaunchKernelGGL((k_tile_forward<T, B, kTileThreads, false, MINB>), dim3(grid), dim3(kTileThreads), 0, st, p,
                       fr, runs, recs, segs, n_segs, n_tb);
  return hipGetLastError();
}

hipError_t launch_tile_forward(int dtype, void* psi, const FrameDesc& fr, const RunDesc* runs, const RunRec* recs,
                               const SegDesc* segs, int n_segs, uint64_t n_tb, int grid, hipStream_t st) {
  if (dtype == 0) return tile_forward_t<double2, kTileSweepC128>(psi, fr, runs, recs, segs, n_segs, n_tb, grid, st);
  if (dtype == 1)
    return tile_forward_t<float2, kTileSweepC64, kSweepBlocks8>(psi, fr, runs, recs, segs, n_segs, n_tb, grid, st);
  return tile_forward_t<R64, kTileSweepR64, kSweepBlocks8>(psi, fr, runs, recs, segs, n_segs, n_tb, grid, st);
}

template <typename T, int B, int GRAD, int MAXS, int MINB>
static hipError_t tile_reverse_g(void* psi, void* lam, const FrameDesc& fr, const RunDesc* runs, const RunRec* recs,
                                 const SegDesc* segs, int n_segs, const uint32_t* slot_map, int n_slots,
                                 double* partials, uint32_t nb, uint64_t n_tb, int grid, const double* imag_count,
                                 hipStream_t st) {
  T* p = static_cast<T*>(psi);
  T* l = static_cast<T*>(lam);
  if (fr.b == B)
    hipLaunchKernelGGL((k_tile_reverse<T, B, kTileThreads, GRAD, MAXS, true, MINB>), dim3(grid), dim3(kTileThreads),
                       0, st, p, l, fr, runs, recs, segs, n_segs, slot_map, n_slots, partials, nb, n_tb, imag_count);
  else
    hipLaunchKernelGGL((k_tile_reverse<T, B, kTileThreads, GRAD, MAXS, false, MINB>), dim3(grid),
                       dim3(kTileThreads), 0, st, p, l, fr, runs, recs, segs, n_segs, slot_map, n_slots, partials, nb,
                       n_tb, imag_count);
  return hipGetLastError();
}

template <typename T, int B, int MAXS = kMaxPassSlots, int MINB = 1>
static hipError_t tile_reverse_t(int grad, void* psi, void* lam, const FrameDesc& fr, const RunDesc* runs,
                                 const RunRec* recs, const SegDesc* segs, int n_segs, const uint32_t* slot_map,
                                 int n_slots, double* partials, uint32_t nb, uint64_t n_tb, int grid,
                                 const double* imag_count, hipStream_t st) {
  if (n_slots > MAXS) return hipErrorInvalidValue;
  if (grad == 0)
    return tile_reverse_g<T, B, 0, 1, MINB>(psi, lam, fr, runs, recs, segs, n_segs, slot_map, n_slots, partials, nb,
                                            n_tb, grid, imag_count, st);
  if (grad == 1)
    return tile_reverse_g<T, B, 1, MAXS, MINB>(psi, lam, fr, runs, recs, segs, n_segs, slot_map, n_slots, partials,
                                               nb, n_tb, grid, imag_count, st);
  return tile_reverse_g<T, B, 2, MAXS, MINB>(psi, lam, fr, runs, recs, segs, n_segs, slot_map, n_slots, partials, nb,
                                             n_tb, grid, imag_count, st);
}

hipError_t launch_tile_reverse(int dtype, int grad, void* psi, void* lam, const FrameDesc& fr,
                               const RunDesc* runs, const RunRec* recs, const SegDesc* segs, int n_segs,
                               const uint32_t* slot_map, int n_slots, double* partials, uint32_t nb_stride,
                               uint64_t n_tb, int grid, const double* imag_count, hipStream_t st) {
  if (n_slots > kMaxPassSlots) return hipErrorInvalidValue;
  if (dtype == 0)
    return tile_reverse_t<double2, kTileTwoC128>(grad, psi, lam, fr, runs, recs, segs, n_segs, slot_map, n_slots,
                                                 partials, nb_stride, n_tb, grid, imag_count, st);
  if (dtype == 1)
    return tile_reverse_t<float2, kTileTwoC64>(grad, psi, lam, fr, runs, recs, segs, n_segs, slot_map, n_slots,
                                               partials, nb_stride, n_tb, grid, imag_count, st);
  return tile_reverse_t<R64, kTileTwoR64>(grad, psi, lam, fr, runs, recs, segs, n_segs, slot_map, n_slots, partials,
                                          nb_stride, n_tb, grid, nullptr, st);
}

}  // namespace q2sv
