// Pauli-sum passes on gfx950 (Section 3.1, Eq. 1-2; lambda = H psi of
// Algorithm 1): the X-grouped expectation and the lambda build over gathered
// LDS tiles, the diagonal part as a resident FP64 vector, and whole-state
// passes for groups whose support does not fit a tile.
//
// Group tables of a tile (TileHdr blob) are copied into LDS once per block.
// In the lambda build every wavefront owns a fixed region of the tile's
// outputs (frame bits wb_mask = its wavefront index), so the groups of a tile
// run with no block barrier between them; only the outputs a group actually
// reaches (its active support patterns) are enumerated.
#include "device_common.h"
#include "launch.h"

namespace q2sv {

struct BlobView {
  const TileHdr* hdr;
  const TGroup* groups;
  const TOut* outs;
  const TSub* subs;
  const double2* coef;
  __device__ explicit BlobView(const uint4* blob) {
    const char* b = reinterpret_cast<const char*>(blob);
    hdr = reinterpret_cast<const TileHdr*>(b);
    groups = reinterpret_cast<const TGroup*>(b + sizeof(TileHdr));
    outs = reinterpret_cast<const TOut*>(b + hdr->off_out);
    subs = reinterpret_cast<const TSub*>(b + hdr->off_sub);
    coef = reinterpret_cast<const double2*>(b + hdr->off_coef);
  }
};

template <int NT>
__device__ __forceinline__ void blob_stage(const uint4* __restrict__ src, uint4* dst) {
  const uint32_t words = reinterpret_cast<const TileHdr*>(src)->bytes / 16;
  for (uint32_t i = threadIdx.x; i < words; i += NT) dst[i] = src[i];
}

// G of one output: sum over subgroups of (-1)^{|m' & w|} T_w[rec], conjugated
// when the output is m'.
__device__ __forceinline__ void group_coef(const BlobView& bv, const TGroup& g, const TOut& o, uint32_t mp,
                                           uint64_t base, double& gre, double& gim) {
  gre = 0.0;
  gim = 0.0;
  for (uint32_t k = 0; k < g.n_sub; ++k) {
    const TSub sd = bv.subs[g.sub_off + k];
    const double2 cv = bv.coef[g.coef_off + k * g.n_rec + o.rec];
    const unsigned sg = parity32(mp & sd.w_loc) ^ parity64(base & sd.w_out);
    gre += sg ? -cv.x : cv.x;
    gim += sg ? -cv.y : cv.y;
  }
  if (o.is_mprime) gim = -gim;
}

// ---------------------------------------------------------------------------
// lambda over one tile: MODE 1 lam = diag * psi + H_tile psi; MODE 2 lam += H_tile psi
// ---------------------------------------------------------------------------
template <typename T, int B, int NT, int MODE>
__global__ void __launch_bounds__(NT) k_tile_lambda(const T* __restrict__ psi, T* __restrict__ lam,
                                                    const double* __restrict__ diag, FrameDesc fr,
                                                    const uint4* __restrict__ blob_g, uint64_t n_tb) {
  using R = typename Real<T>::type;
  constexpr int NW = NT / 64;
  constexpr int PER = (1 << B) / NT;
  constexpr int RPER = ((1 << B) / NW + 63) / 64;
  __shared__ T tp[1 << B];
  __shared__ double2 tl[1 << B];
  __shared__ FrameLut lut;
  __shared__ uint4 blob[kBlobWords];
  blob_stage<NT>(blob_g, blob);
  frame_lut_init<NT>(fr, lut);
  __syncthreads();
  const BlobView bv(blob);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t nloc = 1u << fr.b;
  // this wavefront's output region: frame bits wb_mask equal to `wave`
  const uint32_t wbm = bv.hdr->wb_mask;
  uint64_t wpack = 0;
  int nwb = 0;
  uint32_t wbits = 0;
  for (uint32_t m = wbm; m; m &= m - 1) {
    const int p = __ffs(m) - 1;
    wbits |= uint32_t((wave >> nwb) & 1) << p;
    wpack |= uint64_t(p) << (4 * nwb);
    ++nwb;
  }
  const bool owner = wave < (1 << nwb);
  const uint32_t nreg = nloc >> nwb;
  auto region_l = [&](uint32_t i) { return insert_zeros32_p4(i, wpack, nwb) | wbits; };

  Stage<T, PER> rp;
  Stage<T, RPER> rl;
  double rd[RPER];
  auto fetch = [&](uint64_t tbx) {
    const uint64_t bx = frame_base(fr, tbx);
    tile_fetch<T, PER, NT>(psi, lut, bx, nloc, rp);
    if (owner) {
#pragma unroll
      for (int k = 0; k < RPER; ++k) {
        const uint32_t i = uint32_t(lane) + 64u * k;
        if (i < nreg) {
          const uint64_t gi = bx | frame_deposit(lut, region_l(i));
          if (MODE == 1) {
            rd[k] = diag ? diag[gi] : 0.0;
          } else {
            const T v = lam[gi];
            rl.re[k] = v.x;
            rl.im[k] = v.y;
          }
        }
      }
    }
  };

  uint64_t tb = blockIdx.x;
  if (tb < n_tb) fetch(tb);
  for (; tb < n_tb; tb += gridDim.x) {
    const uint64_t base = frame_base(fr, tb);
    tile_put<T, PER, NT>(tp, nloc, rp);
    __syncthreads();
    if (owner) {
#pragma unroll
      for (int k = 0; k < RPER; ++k) {
        const uint32_t i = uint32_t(lane) + 64u * k;
        if (i < nreg) {
          const uint32_t l = region_l(i);
          double2 v;
          if (MODE == 1) {
            const T a = tp[l];
            v.x = rd[k] * (double)a.x;
            v.y = rd[k] * (double)a.y;
          } else {
            v.x = (double)rl.re[k];
            v.y = (double)rl.im[k];
          }
          tl[l] = v;
        }
      }
    }
    const uint64_t nx = tb + gridDim.x;
    if (nx < n_tb) fetch(nx);
    if (owner) {
      for (uint32_t gi = 0; gi < bv.hdr->n_groups; ++gi) {
        const TGroup g = bv.groups[gi];
        const uint32_t s_wb = g.sup_mask & wbm;
        const int nf = int(fr.b) - int(g.n_ins);
        auto emit = [&](uint32_t ob, uint32_t j) {
          const TOut o = bv.outs[g.out_off + j];
          if ((uint32_t(o.bits) ^ wbits) & s_wb) return;  // pattern lies in another region
          const uint32_t l = ob | o.bits | (wbits & ~g.sup_mask);
          const uint32_t src = l ^ g.x_loc;
          double gre, gim;
          group_coef(bv, g, o, o.is_mprime ? l : src, base, gre, gim);
          const T a = tp[src];
          double2 v = tl[l];
          v.x += gre * (double)a.x - gim * (double)a.y;
          v.y += gre * (double)a.y + gim * (double)a.x;
          tl[l] = v;
        };
        if (nf <= 6) {
          const uint32_t t = uint32_t(lane) & ((1u << nf) - 1u);
          const uint32_t ob = insert_zeros32_p4(t, g.ins_pack, g.n_ins);
          for (uint32_t j = uint32_t(lane) >> nf; j < g.n_out; j += (64u >> nf)) emit(ob, j);
        } else {
          for (uint32_t t = uint32_t(lane); t < (1u << nf); t += 64u) {
            const uint32_t ob = insert_zeros32_p4(t, g.ins_pack, g.n_ins);
            for (uint32_t j = 0; j < g.n_out; ++j) emit(ob, j);
          }
        }
      }
      // the region is complete: write it out
#pragma unroll
      for (int k = 0; k < RPER; ++k) {
        const uint32_t i = uint32_t(lane) + 64u * k;
        if (i < nreg) {
          const uint32_t l = region_l(i);
          const double2 v = tl[l];
          lam[base | frame_deposit(lut, l)] = cmake<T>(R(v.x), R(v.y));
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// expectation over tiles: partials[block] = sum over the tile's groups of
// sum_m conj(psi[m]) (H_x psi)[m], as 2 Re(conj(psi[m]) G psi[m']) per pair.
// Block b works on tile b / bpt; tiles are independent (psi is only read).
// ---------------------------------------------------------------------------
template <typename T, int B, int NT>
__global__ void __launch_bounds__(NT) k_tile_expect(const T* __restrict__ psi, const FrameDesc* __restrict__ frames,
                                                    const uint32_t* __restrict__ blob_off,
                                                    const uint4* __restrict__ blobs, uint32_t bpt, uint64_t n_tb,
                                                    double* __restrict__ partials) {
  constexpr int PER = (1 << B) / NT;
  __shared__ T tp[1 << B];
  __shared__ FrameLut lut;
  __shared__ uint4 blob[kBlobWords];
  __shared__ double red[NT / 64];
  const uint32_t tile = blockIdx.x / bpt, bi = blockIdx.x % bpt;
  const FrameDesc& fr = frames[tile];
  blob_stage<NT>(blobs + blob_off[tile], blob);
  frame_lut_init<NT>(fr, lut);
  __syncthreads();
  const BlobView bv(blob);
  const uint32_t nloc = 1u << fr.b;
  double e = 0.0;
  Stage<T, PER> rp;
  uint64_t tb = bi;
  if (tb < n_tb) tile_fetch<T, PER, NT>(psi, lut, frame_base(fr, tb), nloc, rp);
  for (; tb < n_tb; tb += bpt) {
    const uint64_t base = frame_base(fr, tb);
    tile_put<T, PER, NT>(tp, nloc, rp);
    __syncthreads();
    const uint64_t nx = tb + bpt;
    if (nx < n_tb) tile_fetch<T, PER, NT>(psi, lut, frame_base(fr, nx), nloc, rp);
    for (uint32_t gi = 0; gi < bv.hdr->n_groups; ++gi) {
      const TGroup g = bv.groups[gi];
      const int ns = int(fr.b) - int(g.n_sins);
      const uint32_t np = uint32_t(g.n_rec) << ns;
      for (uint32_t idx = threadIdx.x; idx < np; idx += NT) {
        const uint32_t r = idx >> ns, t = idx & ((1u << ns) - 1u);
        const TOut o = bv.outs[g.out_off + r];  // the first n_rec outputs are the records (m')
        const uint32_t l2 = insert_zeros32_p4(t, g.sins_pack, g.n_sins) | o.bits;
        const uint32_t l = l2 ^ g.x_loc;
        double gre, gim;
        group_coef(bv, g, o, l2, base, gre, gim);  // o is m': conj(G); undo below
        gim = -gim;
        const T a = tp[l], b = tp[l2];
        const double gbr = gre * (double)b.x - gim * (double)b.y, gbi = gre * (double)b.y + gim * (double)b.x;
        e += 2.0 * ((double)a.x * gbr + (double)a.y * gbi);
      }
    }
    __syncthreads();
  }
  const double s = block_sum<NT>(e, red);
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
        u.y += R(gre * b.y + gim * b.x);
        v.x += R(gre * a.x + gim * a.y);
        v.y += R(gre * a.y - gim * a.x);
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
hipError_t launch_tile_lambda(int dtype, bool first, const void* psi, void* lam, const double* diag,
                              const FrameDesc& fr, const uint4* blob, uint64_t n_tb, int grid, hipStream_t st) {
#define Q2SV_TL(T, B, M)                                                                                   \
  hipLaunchKernelGGL((k_tile_lambda<T, B, kLambdaThreads, M>), dim3(grid), dim3(kLambdaThreads), 0, st, \
                     static_cast<const T*>(psi), static_cast<T*>(lam), diag, fr, blob, n_tb)
  if (dtype == 0) {
    if (first) Q2SV_TL(double2, kTileLamC128, 1);
    else Q2SV_TL(double2, kTileLamC128, 2);
  } else {
    if (first) Q2SV_TL(float2, kTileLamC64, 1);
    else Q2SV_TL(float2, kTileLamC64, 2);
  }
#undef Q2SV_TL
  return hipGetLastError();
}

hipError_t launch_tile_expect(int dtype, const void* psi, const FrameDesc* frames, const uint32_t* blob_off,
                              const uint4* blobs, int n_tiles, uint32_t bpt, uint64_t n_tb, double* partials,
                              hipStream_t st) {
  const dim3 grid(uint32_t(n_tiles) * bpt);
  if (dtype == 0)
    hipLaunchKernelGGL((k_tile_expect<double2, kTileFwdC128, kTileThreads>), grid, dim3(kTileThreads), 0, st,
                       static_cast<const double2*>(psi), frames, blob_off, blobs, bpt, n_tb, partials);
  else
    hipLaunchKernelGGL((k_tile_expect<float2, kTileFwdC64, kTileThreads>), grid, dim3(kTileThreads), 0, st,
                       static_cast<const float2*>(psi), frames, blob_off, blobs, bpt, n_tb, partials);
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
#define Q2SV_GF(T, M)                                                                                  \
  hipLaunchKernelGGL((k_group_full<T, M>), dim3(grid), dim3(256), 0, st, static_cast<const T*>(psi), \
                     static_cast<T*>(lam), g, subs, coef, recbits, n, partials)
  if (dtype == 0) {
    if (mode == 0) Q2SV_GF(double2, 0);
    else Q2SV_GF(double2, 2);
  } else {
    if (mode == 0) Q2SV_GF(float2, 0);
    else Q2SV_GF(float2, 2);
  }
#undef Q2SV_GF
  return hipGetLastError();
}

}  // namespace q2sv
