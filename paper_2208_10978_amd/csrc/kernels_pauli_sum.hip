// Pauli-sum passes on gfx950 (Section 3.1, Eq. 1-2; lambda = H psi of
// Algorithm 1): the X-grouped expectation and the lambda build over gathered
// LDS tiles, the diagonal part as a resident FP64 vector, and whole-state
// passes for groups whose support does not fit a tile.
//
// Both read a tile's group tables (projected-sum blobs) in place through
// scalar loads.  Only the pairs a group actually reaches (its active support
// patterns) are enumerated.
#include "device_common.h"
#include "launch.h"

namespace q2sv {

// x * (-1)^s for s in {0, 1}: flips the sign bit
__device__ __forceinline__ double signed_by(double x, unsigned s) {
  return __hiloint2double(__double2hiint(x) ^ int(s << 31), __double2loint(x));
}

// ---------------------------------------------------------------------------
// Projected-sum tables (XHdr blobs, see XBatch): the expectation and lambda
// tilings share them.
// ---------------------------------------------------------------------------
struct XView {
  const XHdr* hdr;
  const XBatch* batches;
  const XItem* items;
  const uint32_t* start;
  const XRec* recs;
  const TSub* subs;
  const double2* coef;
  __device__ explicit XView(const uint4* blob) {
    const char* b = reinterpret_cast<const char*>(blob);
    hdr = reinterpret_cast<const XHdr*>(b);
    batches = reinterpret_cast<const XBatch*>(b + hdr->off_batch);
    items = reinterpret_cast<const XItem*>(b + hdr->off_items);
    start = reinterpret_cast<const uint32_t*>(b + hdr->off_start);
    recs = reinterpret_cast<const XRec*>(b + hdr->off_rec);
    subs = reinterpret_cast<const TSub*>(b + hdr->off_sub);
    coef = reinterpret_cast<const double2*>(b + hdr->off_coef);
  }
};

// (hr, hi) += conj(a) b
template <typename T>
__device__ __forceinline__ void acc_pair(const T& a, const T& b, double& hr, double& hi) {
  const double ax = (double)a.x, bx = (double)b.x;
  if constexpr (is_real_amp<T>) {
    hr = fma(ax, bx, hr);
    (void)hi;
  } else {
    const double ay = (double)a.y, by = (double)b.y;
    hr = fma(ax, bx, fma(ay, by, hr));
    hi = fma(ax, by, fma(-ay, bx, hi));
  }
}

// a with its sign bits XORed with sgn (0 or 0x80000000): -a or a
__device__ __forceinline__ float2 sign_xor(float2 a, uint32_t sgn) {
  return make_float2(__uint_as_float(__float_as_uint(a.x) ^ sgn), __uint_as_float(__float_as_uint(a.y) ^ sgn));
}
__device__ __forceinline__ double sign_xor1(double v, uint32_t sgn) {
  return __hiloint2double(__double2hiint(v) ^ int(sgn), __double2loint(v));
}
__device__ __forceinline__ double2 sign_xor(double2 a, uint32_t sgn) {
  return make_double2(sign_xor1(a.x, sgn), sign_xor1(a.y, sgn));
}
__device__ __forceinline__ R64 sign_xor(R64 a, uint32_t sgn) { return R64{sign_xor1(a.x, sgn)}; }

// An LDS element by byte offset (the tile sits at a fixed LDS address, which
// the read instruction takes as its immediate offset).
template <typename T>
__device__ __forceinline__ T lds_at(const T* tp, uint32_t off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(tp) + off);
}

// lambda over one work item of a batch (the fast build).  Per record each
// lane first forms G at its 2^NR register patterns from the subgroups: one
// signed sum of T_k[r] per class (the signs of the lane's, the record's and
// the out-of-frame bits of w_k), then the butterfly over v, since
// G(v) = sum_cls (-1)^{|v & cls|} A_cls.  G is then the same for every chunk
// but for the chunk's w0 sign.  The chunk walk reads both ends of each pair
// and adds lam[m] += G psi[m'] and lam[m'] += conj(G) psi[m] into the tile's
// fixed-point accumulators (G pre-scaled by the launch's 2^sh, each term
// rounded to an integer by the fused add of kFxMagic) with LDS integer atomic
// adds: other wavefronts may update the same outputs, in any order, and the
// sums do not depend on it.  REAL: psi, T and lambda are real; only real
// parts are read and added.
template <typename TT, bool REAL, int NR, bool MULTI, bool SIGNED>
__device__ __forceinline__ void x_lambda_records(const XView& xv, const XBatch* bp, const XItem& it, uint64_t base,
                                                 const TT* tp, unsigned long long* alr, unsigned long long* ali,
                                                 int sh, uint32_t dl, uint32_t sdl) {
  constexpr int NV = 1 << NR;
  constexpr int NA = MULTI ? NV : 1;
  uint32_t vs[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) vs[v] = bp->vslot[v];
  const uint32_t sx = bp->sx, n_rec = bp->n_rec, rec_off = bp->rec_off;
  const uint32_t n_sub = bp->n_sub, sub_off = bp->sub_off, coef_off = bp->coef_off;
  const uint32_t r1 = it.recs >> 16, c0 = it.chunks & 0xffffu, c1 = it.chunks >> 16;
  for (uint32_t r = it.recs & 0xffffu; r < r1; ++r) {
    const XRec rc = xv.recs[rec_off + r];
    double gr[NA], gi[NA];
#pragma unroll
    for (int v = 0; v < NA; ++v) gr[v] = gi[v] = 0.0;
    uint32_t k0 = 0;
#pragma unroll
    for (int cls = 0; cls < NA; ++cls) {
      const uint32_t k1 = MULTI ? bp->cls_end[cls] : n_sub;
      for (uint32_t k = k0; k < k1; ++k) {
        const TSub sd = xv.subs[sub_off + k];
        const double2 cv = xv.coef[coef_off + k * n_rec + r];
        const unsigned par = unsigned(__popc(dl & sd.w_loc)) + unsigned(__popc(rc.bits & sd.w_loc)) +
                             unsigned(__popcll(base & sd.w_out));
        gr[cls] += signed_by(cv.x, par);
        if constexpr (!REAL) gi[cls] += signed_by(cv.y, par);
      }
      k0 = k1;
    }
    if constexpr (MULTI) {
#pragma unroll
      for (int h = 1; h < NV; h <<= 1)
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (!(v & h)) {
            const double r0 = gr[v], r1v = gr[v | h], i0 = gi[v], i1 = gi[v | h];
            gr[v] = r0 + r1v;
            gr[v | h] = r0 - r1v;
            gi[v] = i0 + i1;
            gi[v | h] = i0 - i1;
          }
    }
#pragma unroll
    for (int v = 0; v < NA; ++v) {
      gr[v] = __builtin_ldexp(gr[v], sh);
      gi[v] = __builtin_ldexp(gi[v], sh);
    }
    const uint32_t lb = sdl ^ rc.slot;
    uint32_t cw = bp->cword[c0];
    for (uint32_t c = c0; c < c1; ++c) {
      const uint32_t cn = c + 1 < c1 ? bp->cword[c + 1] : 0u;  // prefetch
      const uint32_t u = lb ^ (cw & 0x7fffffffu);
      const uint32_t sg = cw & 0x80000000u;
      uint32_t ob[NV];
      TT pm[NV], pp[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        ob[v] = u ^ vs[v];      // m'
        pm[v] = tp[ob[v] ^ sx];  // m = m' ^ x
        pp[v] = tp[ob[v]];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const uint32_t om = ob[v] ^ sx;
        double g_r = gr[MULTI ? v : 0];
        if constexpr (SIGNED) g_r = sign_xor1(g_r, sg);
        if constexpr (REAL) {
          lds_add_fx(&alr[om], fma(g_r, (double)pp[v].x, kFxMagic));     // lam[m] += G psi[m']
          lds_add_fx(&alr[ob[v]], fma(g_r, (double)pm[v].x, kFxMagic));  // lam[m'] += G psi[m]
        } else {
          double g_i = gi[MULTI ? v : 0];
          if constexpr (SIGNED) g_i = sign_xor1(g_i, sg);
          const double ppx = (double)pp[v].x, ppy = (double)pp[v].y, pmx = (double)pm[v].x, pmy = (double)pm[v].y;
          lds_add_fx(&alr[om], fma(g_r, ppx, fma(-g_i, ppy, kFxMagic)));  // lam[m] += G psi[m']
          lds_add_fx(&ali[om], fma(g_r, ppy, fma(g_i, ppx, kFxMagic)));
          lds_add_fx(&alr[ob[v]], fma(g_r, pmx, fma(g_i, pmy, kFxMagic)));  // lam[m'] += conj(G) psi[m]
          lds_add_fx(&ali[ob[v]], fma(g_r, pmy, fma(-g_i, pmx, kFxMagic)));
        }
      }
      cw = cn;
    }
  }
}

template <typename TT, bool REAL, int NR, bool MULTI>
__device__ __forceinline__ void x_lambda_records_s(const XView& xv, const XBatch* bp, const XItem& it, uint64_t base,
                                                   const TT* tp, unsigned long long* alr, unsigned long long* ali,
                                                   int sh, uint32_t dl, uint32_t sdl) {
  if (bp->signed_chunks) x_lambda_records<TT, REAL, NR, MULTI, true>(xv, bp, it, base, tp, alr, ali, sh, dl, sdl);
  else x_lambda_records<TT, REAL, NR, MULTI, false>(xv, bp, it, base, tp, alr, ali, sh, dl, sdl);
}

template <typename TT, bool REAL>
__device__ __forceinline__ void x_lambda_item(const XView& xv, const XItem& it, uint64_t base, const TT* tp,
                                              unsigned long long* alr, unsigned long long* ali, int sh,
                                              uint32_t lane) {
  const XBatch* bp = xv.batches + it.batch;
  const uint32_t lp = bp->lane_pack, nl = bp->n_lane;
  if ((lane >> nl) != 0u) return;  // lanes past a small frame's free bits
  uint32_t dl = 0;
#pragma unroll
  for (int i = 0; i < kXLaneBits; ++i)
    if (uint32_t(i) < nl) dl |= ((lane >> i) & 1u) << ((lp >> (4 * i)) & 15u);
  const uint32_t sdl = lds_swz(dl);
  static_assert(kXRegBits == 2, "one case per register-bit count");
  switch (bp->n_reg + (bp->n_cls > 1 ? 4u : 0u)) {
    case 0: x_lambda_records_s<TT, REAL, 0, false>(xv, bp, it, base, tp, alr, ali, sh, dl, sdl); break;
    case 1: x_lambda_records_s<TT, REAL, 1, false>(xv, bp, it, base, tp, alr, ali, sh, dl, sdl); break;
    case 2: x_lambda_records_s<TT, REAL, 2, false>(xv, bp, it, base, tp, alr, ali, sh, dl, sdl); break;
    case 5: x_lambda_records_s<TT, REAL, 1, true>(xv, bp, it, base, tp, alr, ali, sh, dl, sdl); break;
    case 6: x_lambda_records_s<TT, REAL, 2, true>(xv, bp, it, base, tp, alr, ali, sh, dl, sdl); break;
    default: break;  // several classes need a register bit: not planned
  }
}

// An LDS slot of a real psi tile: the amplitude's real part in FP64.
struct RealSlot {
  double x;
};
template <> struct Real<RealSlot> { using type = double; };

// ---------------------------------------------------------------------------
// lambda over one tile: MODE 1 lam = diag * psi + H_tile psi; MODE 2 lam += H_tile psi
//
// The tile's group tables are projected-sum batches (XBatch) read from global
// memory: every index into them is uniform over a wavefront, so they arrive
// through scalar loads into SGPRs and feed the vector arithmetic directly.
// All wavefronts of the block work on the whole tile at once, each on its
// host-balanced list of work items, and add their terms into 64-bit
// fixed-point accumulators with LDS integer atomic adds (which return
// nothing, so an update is never a load-modify-store chain).  Integer sums do
// not depend on the order in which the updates of different wavefronts
// arrive, so lambda is the same from run to run.
// ---------------------------------------------------------------------------
// The fixed-point exponent s of a lambda launch: the blob's fx_shift minus
// the largest exponent e of |re| + |im| over psi (launch_amp_exponent's
// partials ep[0..n_ep)); with it no term reaches 2^50 and no slot's sum 2^62.
// e is taken as at least -973 (a zero psi gives kFxNone): G 2^s then stays
// below 2^1023, since fx_shift <= 50 - e_g.  red: NT / 64 ints of LDS.  One
// barrier.
template <int NT>
__device__ __forceinline__ int lambda_shift(const uint4* __restrict__ blob, const double* __restrict__ ep, int n_ep,
                                            int* red) {
  int e = kFxNone;
  for (int i = int(threadIdx.x); i < n_ep; i += NT) e = max(e, int(ep[i]));
  e = wave_max_i32(e);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
  __syncthreads();
  int m = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) m = max(m, red[w]);
  return __builtin_amdgcn_readfirstlane(reinterpret_cast<const XHdr*>(blob)->fx_shift - max(m, -973));
}

// The tile passes of a lambda build, on the block's LDS arrays: tp, the psi
// tile of TT slots; alr, ali, 64-bit fixed-point accumulators of lambda's
// real and imaginary parts, cleared per tile, while the tile's starting
// values (diag psi, or the lambda of earlier passes) wait in registers; the
// result is start + accumulator * 2^-sh, sh from lambda_shift.
// REAL: psi and every coefficient are real, so only real parts are read and
// accumulated and ali is not used; TT = RealSlot keeps only the real parts
// of psi in the tile.
template <typename T, int B, int NT, int MODE, bool FULL, bool REAL, typename TT = T>
__device__ __forceinline__ void lambda_tiles(const T* __restrict__ psi, T* __restrict__ lam,
                                             const double* __restrict__ diag, const FrameDesc& fr,
                                             const uint4* __restrict__ blob, uint64_t n_tb, TT* tp,
                                             unsigned long long* alr, unsigned long long* ali, int sh) {
  static_assert(REAL || std::is_same<TT, T>::value, "a real-part tile needs the real build");
  using R = typename Real<T>::type;
  constexpr bool kRealTile = std::is_same<TT, RealSlot>::value;
  constexpr int NW = NT / 64;
  constexpr int PER = (1 << B) / NT;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // every wavefront on the whole tile, on its work list, scale 2^sh
  auto apply_groups = [&](uint64_t base) {
    const XView xv(blob);
    const bool lists = xv.hdr->n_waves == uint32_t(NW);
    const uint32_t i0 = lists ? xv.start[wave] : uint32_t(wave);
    const uint32_t i1 = lists ? xv.start[wave + 1] : xv.hdr->n_items;
    const uint32_t step = lists ? 1u : uint32_t(NW);
    for (uint32_t i = i0; i < i1; i += step)
      x_lambda_item<TT, REAL>(xv, xv.items[i], base, tp, alr, ali, sh, uint32_t(lane));
    __syncthreads();
  };
  // a finished slot: start + accumulator * 2^-sh (the scaling is exact)
  auto result = [&](double start, unsigned long long acc) {
    return start + __builtin_ldexp(double(static_cast<long long>(acc)), -sh);
  };
  // the thread index, opaque to the optimiser: the LDS slots of the staged
  // values are recomputed where they are used instead of being held across
  // the tile loop (where they would spill)
  auto tid_here = []() {
    uint32_t t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
  };

  Stage<T, PER> rp;
  Stage<T, PER> rl;
  double rd[PER];
  double ir[PER], ii[PER];  // the tile's starting values
  uint64_t tb = blockIdx.x;
  if constexpr (FULL) {
    // next loads before the groups; this tile's lambda leaves only after the
    // next tile is in place, so its stores overlap the next tile's groups
    const TileAddrLean<NT, PER> ta(fr);
    auto fetch = [&](uint64_t bx) {
      tile_fetch_full<T, PER, NT>(psi, ta, fr, bx, rp);
      if (MODE == 1) {
        if (diag) {
          const double* d = diag + bx;
#pragma unroll
          for (int i = 0; i < PER; ++i) rd[i] = d[lean_off(ta, fr, i)];
        } else {
#pragma unroll
          for (int i = 0; i < PER; ++i) rd[i] = 0.0;
        }
      } else {
        tile_fetch_full<T, PER, NT>(lam, ta, fr, bx, rl);
      }
    };
    auto put = [&]() {
      const uint32_t tid = tid_here();
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        if constexpr (kRealTile) tp[lds_swz(tid + uint32_t(i) * NT)].x = double(rp.re[i]);
        else tp[lds_swz(tid + uint32_t(i) * NT)] = cmake<T>(rp.re[i], rp.im[i]);
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const uint32_t sl = lds_swz(tid + uint32_t(i) * NT);
        ir[i] = MODE == 1 ? rd[i] * (double)rp.re[i] : (double)rl.re[i];
        ii[i] = REAL ? 0.0 : MODE == 1 ? rd[i] * (double)rp.im[i] : (double)rl.im[i];
        alr[sl] = 0ull;
        if (!REAL) ali[sl] = 0ull;
      }
    };
    if (tb < n_tb) {
      fetch(frame_base(fr, tb));
      put();
    }
    __syncthreads();
    for (; tb < n_tb; tb += gridDim.x) {
      const uint64_t base = frame_base(fr, tb);
      const uint64_t nx = tb + gridDim.x;
      if (nx < n_tb) fetch(frame_base(fr, nx));
      apply_groups(base);
      Stage<T, PER> out;
      const uint32_t tid = tid_here();
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const uint32_t sl = lds_swz(tid + uint32_t(i) * NT);
        out.re[i] = R(result(ir[i], alr[sl]));
        out.im[i] = REAL ? R(0) : R(result(ii[i], ali[sl]));
      }
      if (nx < n_tb) put();
      tile_send<T, PER, NT>(lam, ta, fr, base, out);
      __syncthreads();
    }
  } else {
    __shared__ FrameLut lut;
    frame_lut_init<NT>(fr, lut);
    __syncthreads();
    const uint32_t nloc = 1u << fr.b;
    auto fetch = [&](uint64_t tbx) {
      const uint64_t bx = frame_base(fr, tbx);
      tile_fetch<T, PER, NT>(psi, lut, bx, nloc, rp);
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const uint32_t l = threadIdx.x + uint32_t(i) * NT;
        if (l < nloc) {
          const uint64_t gi = bx | frame_deposit(lut, l);
          if (MODE == 1) {
            rd[i] = diag ? diag[gi] : 0.0;
          } else {
            const T v = lam[gi];
            rl.re[i] = v.x;
            rl.im[i] = v.y;
          }
        }
      }
    };
    if (tb < n_tb) fetch(tb);
    for (; tb < n_tb; tb += gridDim.x) {
      const uint64_t base = frame_base(fr, tb);
      if constexpr (kRealTile) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
          const uint32_t l = threadIdx.x + uint32_t(i) * NT;
          if (l < nloc) tp[lds_swz(l)].x = double(rp.re[i]);
        }
      } else {
        tile_put<T, PER, NT>(tp, nloc, rp);
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const uint32_t l = threadIdx.x + uint32_t(i) * NT;
        if (l < nloc) {
          const uint32_t sl = lds_swz(l);
          ir[i] = MODE == 1 ? rd[i] * (double)rp.re[i] : (double)rl.re[i];
          ii[i] = REAL ? 0.0 : MODE == 1 ? rd[i] * (double)rp.im[i] : (double)rl.im[i];
          alr[sl] = 0ull;
          if (!REAL) ali[sl] = 0ull;
        }
      }
      __syncthreads();
      const uint64_t nx = tb + gridDim.x;
      if (nx < n_tb) fetch(nx);
      apply_groups(base);
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const uint32_t l = threadIdx.x + uint32_t(i) * NT;
        if (l < nloc) {
          const uint32_t sl = lds_swz(l);
          const double vr = result(ir[i], alr[sl]);
          const double vi = REAL ? 0.0 : result(ii[i], ali[sl]);
          lam[base | frame_deposit(lut, l)] = cmake<T>(R(vr), R(vi));
        }
      }
    }
  }
}

// lambda = H psi over the tiles of one frame.  MODE 1 starts from the
// diagonal part, MODE 2 adds to lam.
template <typename T, int B, int NT, int MODE, bool FULL>
__global__ void __launch_bounds__(NT) k_tile_lambda(const T* __restrict__ psi, T* __restrict__ lam,
                                                    const double* __restrict__ diag, FrameDesc fr,
                                                    const uint4* __restrict__ blob, uint64_t n_tb,
                                                    const double* __restrict__ ep, int n_ep) {
  __shared__ T tp[1 << B];
  __shared__ unsigned long long alr[1 << B], ali[1 << B];
  __shared__ int red[NT / 64];
  const int sh = lambda_shift<NT>(blob, ep, n_ep, red);
  lambda_tiles<T, B, NT, MODE, FULL, false>(psi, lam, diag, fr, blob, n_tb, tp, alr, ali, sh);
}

// The same for a real psi and a sum with real coefficients: lambda is real,
// the tile keeps psi's real parts (8 bytes a slot) and one FP64 accumulator,
// so a frame holds one qubit more in the same LDS; lam's imaginary parts are
// written as zero.
//
// guard (device, may be NULL): the number of psi's nonzero imaginary parts,
// given when the real build was chosen on the caller's word rather than on
// that count.  If it is not zero the caller's word was wrong: the pass
// writes NaN over its tiles of lambda instead, so the energy and gradient
// computed from it are NaN rather than silently wrong.
template <typename T, int NT>
__device__ __forceinline__ void lambda_poison(T* __restrict__ lam, const FrameDesc& fr, uint64_t n_tb) {
  using R = typename Real<T>::type;
  const R nan = R(__builtin_nan(""));
  const uint32_t nloc = 1u << fr.b;
  for (uint64_t tb = blockIdx.x; tb < n_tb; tb += gridDim.x) {
    const uint64_t base = frame_base(fr, tb);
    for (uint32_t l = threadIdx.x; l < nloc; l += NT) {
      uint64_t g = 0;
      for (int j = 0; j < int(fr.b); ++j)
        if ((l >> j) & 1u) g |= uint64_t(1) << fr.q[j];
      lam[base | g] = cmake<T>(nan, nan);
    }
  }
}

template <typename T, int B, int NT, int MODE, bool FULL>
__global__ void __launch_bounds__(NT) k_tile_lambda_real(const T* __restrict__ psi, T* __restrict__ lam,
                                                         const double* __restrict__ diag, FrameDesc fr,
                                                         const uint4* __restrict__ blob, uint64_t n_tb,
                                                         const double* __restrict__ guard,
                                                         const double* __restrict__ ep, int n_ep) {
  __shared__ RealSlot tp[1 << B];
  __shared__ unsigned long long alr[1 << B];
  __shared__ int red[NT / 64];
  if (guard && *guard != 0.0) {
    lambda_poison<T, NT>(lam, fr, n_tb);
    return;
  }
  const int sh = lambda_shift<NT>(blob, ep, n_ep, red);
  lambda_tiles<T, B, NT, MODE, FULL, true, RealSlot>(psi, lam, diag, fr, blob, n_tb, tp, alr, nullptr, sh);
}

// ---------------------------------------------------------------------------
// Expectation over one tile (projected sums, see XBatch).  The tile's groups
// come in batches; wavefront w takes the batches of its work list (balanced
// on the host) and, for each record, sums P = conj(psi[m]) psi[m'] over the
// batch's pairs into one FP64 accumulator per register pattern v: per pair
// two LDS reads, the slot arithmetic and four FMAs (plus the conversions of
// complex64), whatever the number of subgroups.  The subgroups then take
// their sums from the Walsh-Hadamard transform of the accumulators, with the
// sign of their lane, record and out-of-frame bits; each lane keeps its FP64
// sum, reduced per block in a fixed order.
// ---------------------------------------------------------------------------
// One work item of a batch: NR register bits (2^NR positions per lane and
// chunk); MULTI: subgroups of several classes (one accumulator per v), else
// every subgroup has class 0 and one accumulator takes every position;
// SIGNED: some chunk words carry the sign of w0 on their bits (the first
// amplitude of the pair is negated in its raw bits), else none do.  Slots
// travel as byte offsets (slot * sizeof(T); the map stays linear), and the
// next chunk word is fetched while the current chunk is summed.
template <typename T, int NR, bool MULTI, bool SIGNED>
__device__ __forceinline__ double x_records(const XView& xv, const XBatch* bp, const XItem& it, uint64_t base,
                                            const T* tp, uint32_t dl, uint32_t sdl) {
  constexpr int NV = 1 << NR;
  constexpr int NA = MULTI ? NV : 1;
  constexpr int LG = ilog2c(sizeof(T));
  uint32_t vs[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) vs[v] = bp->vslot[v] << LG;
  const uint32_t sx = bp->sx << LG, n_rec = bp->n_rec, rec_off = bp->rec_off;
  const uint32_t n_sub = bp->n_sub, sub_off = bp->sub_off, coef_off = bp->coef_off;
  const uint32_t r1 = it.recs >> 16, c0 = it.chunks & 0xffffu, c1 = it.chunks >> 16;
  const uint32_t sdl_b = sdl << LG;
  double e = 0.0;
  for (uint32_t r = it.recs & 0xffffu; r < r1; ++r) {
    const XRec rc = xv.recs[rec_off + r];
    const uint32_t lb = sdl_b ^ (rc.slot << LG);
    double hr[NA], hi[NA];
#pragma unroll
    for (int v = 0; v < NA; ++v) hr[v] = hi[v] = 0.0;
    uint32_t cw = bp->cword[c0];
    for (uint32_t c = c0; c < c1; ++c) {
      const uint32_t cn = c + 1 < c1 ? bp->cword[c + 1] : 0u;  // prefetch
      const uint32_t u = lb ^ ((cw & 0x7fffffffu) << LG);
      const uint32_t sg = cw & 0x80000000u;
      T a[NV], b[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const uint32_t ob = u ^ vs[v];  // m'
        a[v] = lds_at(tp, ob ^ sx);     // m = m' ^ x
        b[v] = lds_at(tp, ob);
      }
      // every read of the chunk in flight before the arithmetic starts
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if constexpr (SIGNED) a[v] = sign_xor(a[v], sg);
        acc_pair(a[v], b[v], hr[MULTI ? v : 0], hi[MULTI ? v : 0]);
      }
      cw = cn;
    }
    if constexpr (MULTI) {
#pragma unroll
      for (int h = 1; h < NV; h <<= 1)
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (!(v & h)) {
            const double r0 = hr[v], r1v = hr[v | h], i0 = hi[v], i1 = hi[v | h];
            hr[v] = r0 + r1v;
            hr[v | h] = r0 - r1v;
            hi[v] = i0 + i1;
            hi[v | h] = i0 - i1;
          }
    }
    uint32_t k0 = 0;
#pragma unroll
    for (int cls = 0; cls < NA; ++cls) {
      const uint32_t k1 = MULTI ? bp->cls_end[cls] : n_sub;
      for (uint32_t k = k0; k < k1; ++k) {
        const TSub sd = xv.subs[sub_off + k];
        const double2 cv = xv.coef[coef_off + k * n_rec + r];
        const unsigned par = unsigned(__popc(dl & sd.w_loc)) + unsigned(__popc(rc.bits & sd.w_loc)) +
                             unsigned(__popcll(base & sd.w_out));
        double t = cv.x * hr[cls];
        if constexpr (!is_real_amp<T>) t = fma(-cv.y, hi[cls], t);
        e += signed_by(t, par);
      }
      k0 = k1;
    }
  }
  return e;
}

template <typename T, int NR, bool MULTI>
__device__ __forceinline__ double x_records_s(const XView& xv, const XBatch* bp, const XItem& it, uint64_t base,
                                              const T* tp, uint32_t dl, uint32_t sdl) {
  return bp->signed_chunks ? x_records<T, NR, MULTI, true>(xv, bp, it, base, tp, dl, sdl)
                           : x_records<T, NR, MULTI, false>(xv, bp, it, base, tp, dl, sdl);
}

template <typename T>
__device__ __forceinline__ double x_item(const XView& xv, const XItem& it, uint64_t base, const T* tp, uint32_t lane) {
  const XBatch* bp = xv.batches + it.batch;
  const uint32_t lp = bp->lane_pack, nl = bp->n_lane;
  uint32_t dl = 0;
#pragma unroll
  for (int i = 0; i < kXLaneBits; ++i)
    if (uint32_t(i) < nl) dl |= ((lane >> i) & 1u) << ((lp >> (4 * i)) & 15u);
  const uint32_t sdl = lds_swz(dl);
  double e = 0.0;
  static_assert(kXRegBits == 2, "one case per register-bit count");
  switch (bp->n_reg + (bp->n_cls > 1 ? 4u : 0u)) {
    case 0: e = x_records_s<T, 0, false>(xv, bp, it, base, tp, dl, sdl); break;
    case 1: e = x_records_s<T, 1, false>(xv, bp, it, base, tp, dl, sdl); break;
    case 2: e = x_records_s<T, 2, false>(xv, bp, it, base, tp, dl, sdl); break;
    case 5: e = x_records_s<T, 1, true>(xv, bp, it, base, tp, dl, sdl); break;
    case 6: e = x_records_s<T, 2, true>(xv, bp, it, base, tp, dl, sdl); break;
    default: break;  // several classes need a register bit: not planned
  }
  return (lane >> nl) == 0u ? e : 0.0;  // lanes past a small frame's free bits
}

template <typename T, int B, int NT, bool FULL>
__global__ void __launch_bounds__(NT) k_tile_expect(const T* __restrict__ psi, FrameDesc fr,
                                                    const uint4* __restrict__ blob, uint64_t n_tb,
                                                    double* __restrict__ partials) {
  constexpr int NW = NT / 64;
  constexpr int PER = (1 << B) / NT;
  __shared__ T tp[1 << B];
  __shared__ double red[NW];
  const XView xv(blob);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // the host balanced the work lists for NW wavefronts; any other count
  // takes the items round robin
  const bool lists = xv.hdr->n_waves == uint32_t(NW);
  const uint32_t i0 = lists ? xv.start[wave] : wave;
  const uint32_t i1 = lists ? xv.start[wave + 1] : xv.hdr->n_items;
  const uint32_t step = lists ? 1u : uint32_t(NW);
  double e = 0.0;
  auto apply_groups = [&](uint64_t base) {
    for (uint32_t i = i0; i < i1; i += step) e += x_item<T>(xv, xv.items[i], base, tp, lane);
    __syncthreads();
  };
  Stage<T, PER> rp;
  uint64_t tb = blockIdx.x;
  if constexpr (FULL) {
    const TileAddrLean<NT, PER> ta(fr);
    if (tb < n_tb) tile_fetch_full<T, PER, NT>(psi, ta, fr, frame_base(fr, tb), rp);
    for (; tb < n_tb; tb += gridDim.x) {
      const uint64_t base = frame_base(fr, tb);
      tile_put_full<T, PER, NT>(tp, rp);
      __syncthreads();
      const uint64_t nx = tb + gridDim.x;
      if (nx < n_tb) tile_fetch_full<T, PER, NT>(psi, ta, fr, frame_base(fr, nx), rp);
      apply_groups(base);
    }
  } else {
    __shared__ FrameLut lut;
    frame_lut_init<NT>(fr, lut);
    __syncthreads();
    const uint32_t nloc = 1u << fr.b;
    if (tb < n_tb) tile_fetch<T, PER, NT>(psi, lut, frame_base(fr, tb), nloc, rp);
    for (; tb < n_tb; tb += gridDim.x) {
      const uint64_t base = frame_base(fr, tb);
      tile_put<T, PER, NT>(tp, nloc, rp);
      __syncthreads();
      const uint64_t nx = tb + gridDim.x;
      if (nx < n_tb) tile_fetch<T, PER, NT>(psi, lut, frame_base(fr, nx), nloc, rp);
      apply_groups(base);
    }
  }
  const double s = block_sum<NT>(2.0 * e, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// resident diagonal: d[m] = sum_t c_t (-1)^{|m & z_t|} over the x = 0 terms
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_diag_build(double* __restrict__ d, uint64_t n_amp,
                                                    const uint64_t* __restrict__ z, const double* __restrict__ c,
                                                    int n_terms) {
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  for (uint64_t m = uint64_t(blockIdx.x) * 256 + threadIdx.x; m < n_amp; m += stride) {
    double s = 0.0;
    for (int t = 0; t < n_terms; ++t) s += parity64(m & z[t]) ? -c[t] : c[t];
    d[m] = s;
  }
}

// ---------------------------------------------------------------------------
// one group over the whole state (support too wide for a tile).
// MODE 0: expectation partials; MODE 2: lam += H_x psi in place.
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_group_full(const T* __restrict__ psi, T* __restrict__ lam, GroupDesc g,
                                                    const SubDesc* __restrict__ subs,
                                                    const double2* __restrict__ coef,
                                                    const uint64_t* __restrict__ recbits, int n,
                                                    double* __restrict__ partials) {
  using R = typename Real<T>::type;
  __shared__ double red[4];
  const uint64_t stride = uint64_t(gridDim.x) * 256;
  const uint64_t tid0 = uint64_t(blockIdx.x) * 256 + threadIdx.x;
  double e = 0.0;
  const uint64_t np = g.enumerated ? (uint64_t(1) << (n - g.n_sup)) : (uint64_t(1) << (n - 1));
  for (int r = 0; r < g.n_rec; ++r) {
    const uint64_t bits = g.enumerated ? recbits[g.rec_off + r] : 0ull;
    for (uint64_t t = tid0; t < np; t += stride) {
      uint64_t l2, l;
      if (g.enumerated) {
        l2 = insert_zeros(t, g.sup_pack, g.n_sup) | bits;
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
        T u = lam[l], v = lam[l2];
        u.x += R(gre * b.x - gim * b.y);
        v.x += R(gre * a.x + gim * a.y);
        if constexpr (!is_real_amp<T>) {  // a real state takes real sums only
          u.y += R(gre * b.y + gim * b.x);
          v.y += R(gre * a.y - gim * a.x);
        }
        lam[l] = u;
        lam[l2] = v;
      }
    }
  }
  if (MODE == 0) {
    const double s = block_sum<256>(e, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int B, int M, bool RT>
static void tile_lambda_t(const void* psi, void* lam, const double* diag, const FrameDesc& fr, const uint4* blob,
                          uint64_t n_tb, int grid, const double* guard, const double* ep, int n_ep, hipStream_t st) {
  constexpr int NT = kLambdaThreads;
  const T* p = static_cast<const T*>(psi);
  T* l = static_cast<T*>(lam);
  if constexpr (RT) {
    if (fr.b == B)
      hipLaunchKernelGGL((k_tile_lambda_real<T, B, NT, M, true>), dim3(grid), dim3(NT), 0, st, p, l, diag, fr, blob,
                         n_tb, guard, ep, n_ep);
    else
      hipLaunchKernelGGL((k_tile_lambda_real<T, B, NT, M, false>), dim3(grid), dim3(NT), 0, st, p, l, diag, fr, blob,
                         n_tb, guard, ep, n_ep);
  } else {
    if (fr.b == B)
      hipLaunchKernelGGL((k_tile_lambda<T, B, NT, M, true>), dim3(grid), dim3(NT), 0, st, p, l, diag, fr, blob, n_tb,
                         ep, n_ep);
    else
      hipLaunchKernelGGL((k_tile_lambda<T, B, NT, M, false>), dim3(grid), dim3(NT), 0, st, p, l, diag, fr, blob, n_tb,
                         ep, n_ep);
  }
}

template <typename T, int B, bool RT>
static void tile_lambda_m(bool first, const void* psi, void* lam, const double* diag, const FrameDesc& fr,
                          const uint4* blob, uint64_t n_tb, int grid, const double* guard, const double* ep, int n_ep,
                          hipStream_t st) {
  if (first) tile_lambda_t<T, B, 1, RT>(psi, lam, diag, fr, blob, n_tb, grid, guard, ep, n_ep, st);
  else tile_lambda_t<T, B, 2, RT>(psi, lam, diag, fr, blob, n_tb, grid, guard, ep, n_ep, st);
}

hipError_t launch_tile_lambda(int dtype, bool first, bool real, const void* psi, void* lam, const double* diag,
                              const FrameDesc& fr, const uint4* blob, uint64_t n_tb, int grid, const double* guard,
                              const double* ep, int n_ep, hipStream_t st) {
  if (n_ep < 1 || n_ep > kLambdaThreads) return hipErrorInvalidValue;
  if (dtype == 2) {  // a real state: always the real-part build
    tile_lambda_m<R64, kTileLamReal, true>(first, psi, lam, diag, fr, blob, n_tb, grid, nullptr, ep, n_ep, st);
  } else if (dtype == 0) {
    if (real) tile_lambda_m<double2, kTileLamReal, true>(first, psi, lam, diag, fr, blob, n_tb, grid, guard, ep, n_ep, st);
    else tile_lambda_m<double2, kTileLamC128, false>(first, psi, lam, diag, fr, blob, n_tb, grid, guard, ep, n_ep, st);
  } else {
    if (real) tile_lambda_m<float2, kTileLamReal, true>(first, psi, lam, diag, fr, blob, n_tb, grid, guard, ep, n_ep, st);
    else tile_lambda_m<float2, kTileLamC64, false>(first, psi, lam, diag, fr, blob, n_tb, grid, guard, ep, n_ep, st);
  }
  return hipGetLastError();
}

template <typename T, int B>
static void tile_expect_t(const void* psi, const FrameDesc& fr, const uint4* blob, uint64_t n_tb, int grid,
                          double* partials, hipStream_t st) {
  const T* p = static_cast<const T*>(psi);
  if (fr.b == B)
    hipLaunchKernelGGL((k_tile_expect<T, B, kExpectThreads, true>), dim3(grid), dim3(kExpectThreads), 0, st, p, fr,
                       blob, n_tb, partials);
  else
    hipLaunchKernelGGL((k_tile_expect<T, B, kExpectThreads, false>), dim3(grid), dim3(kExpectThreads), 0, st, p, fr,
                       blob, n_tb, partials);
}

hipError_t launch_tile_expect(int dtype, const void* psi, const FrameDesc& fr, const uint4* blob, uint64_t n_tb,
                              int grid, double* partials, hipStream_t st) {
  if (dtype == 0) tile_expect_t<double2, kTileFwdC128>(psi, fr, blob, n_tb, grid, partials, st);
  else if (dtype == 1) tile_expect_t<float2, kTileFwdC64>(psi, fr, blob, n_tb, grid, partials, st);
  else tile_expect_t<R64, kTileFwdC64>(psi, fr, blob, n_tb, grid, partials, st);
  return hipGetLastError();
}

hipError_t launch_diag_build(double* d, uint64_t n_amp, const uint64_t* z, const double* c, int n_terms,
                             hipStream_t st) {
  const uint64_t want = (n_amp + 255) / 256;
  const int grid = int(want < 8192 ? (want ? want : 1) : 8192);
  hipLaunchKernelGGL(k_diag_build, dim3(grid), dim3(256), 0, st, d, n_amp, z, c, n_terms);
  return hipGetLastError();
}

hipError_t launch_group_full(int dtype, int mode, const void* psi, void* lam, const GroupDesc& g,
                             const SubDesc* subs, const double2* coef, const uint64_t* recbits, int n, int grid,
                             double* partials, hipStream_t st) {
  return by_dtype(dtype, [&](auto tag) {
    using T = decltype(tag);
    if (mode == 0)
      hipLaunchKernelGGL((k_group_full<T, 0>), dim3(grid), dim3(256), 0, st, static_cast<const T*>(psi),
                         static_cast<T*>(lam), g, subs, coef, recbits, n, partials);
    else
      hipLaunchKernelGGL((k_group_full<T, 2>), dim3(grid), dim3(256), 0, st, static_cast<const T*>(psi),
                         static_cast<T*>(lam), g, subs, coef, recbits, n, partials);
  });
}

}  // namespace q2sv
