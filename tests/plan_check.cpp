// Host checks of the tile-walk planning (CPU only, built with the host
// compiler against plan.cpp).  For seeded Jordan-Wigner-shaped rotation lists
// (forward, per-parameter and per-string reverse schedules) every walk must
//   * split the bits its run leaves free (not enumerated, not region bits)
//     into at most six lane bits and the loop bits hi_mask, disjointly;
//   * visit each of the 2^walk_log free-bit patterns exactly once;
//   * carry the LDS slot of each lane bit and its z (or w) parity bit;
//   * use lane bits whose bank-conflict cost (largest number of lanes on one
//     bank word: 16 lanes for 8-byte words, 8 lanes for 16-byte words, the
//     latter weighted by one half) is the least over every ordered choice of
//     free bits for lane bits 0..3;
// and the projected-sum tilings must reproduce the expectation and lambda of
// seeded sums when walked on the CPU as the tile kernels walk them, lambda
// also in the kernels' fixed point (check_expect).
// Prints "ok ..." and exits 0, or names the first failure and exits 1.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <vector>

#include "plan.h"

using namespace q2sv;

static uint64_t g_state = 0x2208109780ull;
static uint64_t next_u64() {  // splitmix64
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static double next_unit() { return double(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

static int g_fail = 0;
static long g_moved = 0;  // run pairs the schedules reordered
#define CHECK(cond, ...)                          \
  do {                                            \
    if (!(cond)) {                                \
      if (g_fail < 10) {                          \
        std::printf("FAIL %s: ", #cond);          \
        std::printf(__VA_ARGS__);                 \
        std::printf("\n");                        \
      }                                           \
      ++g_fail;                                   \
    }                                             \
  } while (0)

// Largest number of the first 2^nl lanes sharing a bank word, by counting.
static int lanes_per_word(const uint32_t* q, int nl, int mod) {
  std::vector<int> cnt(mod, 0);
  int mx = 0;
  for (uint32_t l = 0; l < (1u << nl); ++l) {
    uint32_t s = 0;
    for (int i = 0; i < nl; ++i)
      if ((l >> i) & 1u) s ^= q[i];
    mx = std::max(mx, ++cnt[s % uint32_t(mod)]);
  }
  return mx;
}
static double walk_cost(const uint32_t* lane_bits, int head) {
  uint32_t q[4] = {0, 0, 0, 0};
  for (int i = 0; i < head; ++i) q[i] = lds_slot(lane_bits[i]);
  return double(lanes_per_word(q, head, 16)) + 0.5 * double(lanes_per_word(q, std::min(head, 3), 8));
}
// least cost over every ordered choice of min(4, |free|) free bits
static double best_cost(uint32_t free_bits) {
  static std::map<uint32_t, double> memo;
  auto it = memo.find(free_bits);
  if (it != memo.end()) return it->second;
  std::vector<uint32_t> c;
  for (uint32_t m = free_bits; m; m &= m - 1) c.push_back(m & (~m + 1u));
  const int k = int(c.size()), head = std::min(k, 4);
  double best = 1e30;
  // odometer over ordered tuples of distinct indices
  std::vector<int> cur(head, 0);
  while (true) {
    std::set<int> seen(cur.begin(), cur.end());
    if (int(seen.size()) == head) {
      uint32_t lb[4];
      for (int i = 0; i < head; ++i) lb[i] = c[cur[i]];
      best = std::min(best, walk_cost(lb, head));
    }
    int d = head - 1;
    while (d >= 0 && ++cur[d] == k) cur[d--] = 0;
    if (d < 0) break;
  }
  if (head == 0) best = 0.0;
  memo[free_bits] = best;
  return best;
}

static uint32_t deposit(uint32_t v, uint32_t mask) {
  uint32_t r = 0;
  for (uint32_t m = mask; m; m &= m - 1, v >>= 1)
    if (v & 1u) r |= m & (~m + 1u);
  return r;
}

// Common walk checks; parity_src is z0_loc (rotations) or w_loc (lambda) and
// parity_lanes the lane mask the planner stored for it.
// Every run is scheduled exactly once, and any two runs that the schedule
// applies in the other order than the list (reversed for the reverse sweep)
// commute, checked string by string.
static void check_order(const char* what, const std::vector<Run>& runs, const std::vector<Pass>& passes,
                        const PauliIn* p, bool reverse) {
  const int R = int(runs.size());
  std::vector<int> pos(size_t(R), -1);
  int k = 0;
  for (const Pass& ps : passes)
    for (int ri : ps.runs) {
      CHECK(ri >= 0 && ri < R && pos[size_t(ri)] < 0, "%s: run %d scheduled twice", what, ri);
      pos[size_t(ri)] = k++;
    }
  CHECK(k == R, "%s: %d of %d runs scheduled", what, k, R);
  long moved = 0;
  for (int i = 0; i < R; ++i)
    for (int j = i + 1; j < R; ++j) {
      const int a = reverse ? R - 1 - i : i, b2 = reverse ? R - 1 - j : j;  // a is applied first in the list
      if (pos[size_t(a)] < pos[size_t(b2)]) continue;
      ++moved;
      for (int u = 0; u < runs[size_t(a)].count; ++u)
        for (int v = 0; v < runs[size_t(b2)].count; ++v) {
          const PauliIn& s1 = p[runs[size_t(a)].first + u];
          const PauliIn& s2 = p[runs[size_t(b2)].first + v];
          CHECK(((__builtin_popcountll(s1.x & s2.z) + __builtin_popcountll(s1.z & s2.x)) & 1) == 0,
                "%s: runs %d and %d swapped but do not commute", what, a, b2);
        }
    }
  g_moved += moved;
}

static void check_walk(const char* what, uint32_t free_bits, uint32_t walk_log, const uint32_t* dep_p,
                       const uint32_t* dep_q, uint32_t hi_mask, uint32_t parity_src, uint32_t parity_lanes,
                       long* n_walks, double* cost_sum, double* best_sum) {
  ++*n_walks;
  CHECK(walk_log == uint32_t(__builtin_popcount(free_bits)), "%s walk_log %u free %x", what, walk_log, free_bits);
  const int nl = std::min<int>(int(walk_log), kWalkLaneBits);
  uint32_t lanes = 0;
  for (int i = 0; i < kWalkLaneBits; ++i) {
    if (i < nl) {
      CHECK(dep_p[i] && !(dep_p[i] & (dep_p[i] - 1)), "%s lane bit %d = %x is not one bit", what, i, dep_p[i]);
      CHECK(!(lanes & dep_p[i]), "%s lane bit %d repeats", what, i);
      CHECK(dep_q[i] == lds_slot(dep_p[i]), "%s slot of lane bit %d", what, i);
      CHECK(((parity_lanes >> i) & 1u) == ((parity_src & dep_p[i]) ? 1u : 0u), "%s parity lane %d", what, i);
      lanes |= dep_p[i];
    } else {
      CHECK(dep_p[i] == 0 && dep_q[i] == 0, "%s unused lane bit %d set", what, i);
    }
  }
  CHECK(!(lanes & hi_mask), "%s lane and loop bits overlap", what);
  CHECK((lanes | hi_mask) == free_bits, "%s lanes %x | loop %x != free %x", what, lanes, hi_mask, free_bits);
  // every free-bit pattern exactly once
  if (walk_log <= 14) {
    std::vector<uint8_t> hit(size_t(1) << walk_log, 0);
    const uint32_t nj = 1u << (walk_log - uint32_t(nl));
    bool ok = true;
    for (uint32_t j = 0; j < nj && ok; ++j)
      for (uint32_t l = 0; l < (1u << nl); ++l) {
        uint32_t pos = deposit(j, hi_mask);
        for (int i = 0; i < nl; ++i)
          if ((l >> i) & 1u) pos |= dep_p[i];
        if (pos & ~free_bits) {
          ok = false;
          break;
        }
        // compress pos onto free_bits to index hit[]
        uint32_t idx = 0, k = 0;
        for (uint32_t m = free_bits; m; m &= m - 1, ++k)
          if (pos & m & (~m + 1u)) idx |= 1u << k;
        if (hit[idx]++) ok = false;
      }
    CHECK(ok, "%s walk visits a pattern twice or leaves the free bits", what);
  }
  const int head = std::min(nl, 4);
  const double c = walk_cost(dep_p, head), b = best_cost(free_bits);
  CHECK(c <= b + 1e-12, "%s lane-bit cost %.2f above the least %.2f (free %x)", what, c, b, free_bits);
  *cost_sum += c;
  *best_sum += b;
}

// Jordan-Wigner strings of the singles and doubles of n spin orbitals with
// n_occ occupied: the Y placements with an odd count, Z on the orbitals
// strictly between each creation/annihilation pair.  One parameter per
// excitation.
static void uccsd_like(int n, int n_occ, std::vector<PauliIn>& p, std::vector<int32_t>& param) {
  auto chain = [](int lo, int hi) {
    uint64_t z = 0;
    for (int q = lo + 1; q < hi; ++q) z |= uint64_t(1) << q;
    return z;
  };
  int32_t k = 0;
  for (int i = 0; i < n_occ; ++i)
    for (int a = n_occ; a < n; ++a, ++k) {
      const int idx[2] = {i, a};
      for (int y = 0; y < 2; ++y) {
        const uint64_t x = (uint64_t(1) << i) | (uint64_t(1) << a);
        p.push_back({x, chain(i, a) | (uint64_t(1) << idx[y])});
        param.push_back(k);
      }
    }
  for (int i = 0; i < n_occ; ++i)
    for (int j = i + 1; j < n_occ; ++j)
      for (int a = n_occ; a < n; ++a)
        for (int b = a + 1; b < n; ++b, ++k) {
          const int idx[4] = {i, j, a, b};
          const uint64_t x = (uint64_t(1) << i) | (uint64_t(1) << j) | (uint64_t(1) << a) | (uint64_t(1) << b);
          for (uint32_t ys = 0; ys < 16; ++ys) {
            if (!(__builtin_popcount(ys) & 1)) continue;
            uint64_t z = chain(i, j) | chain(a, b);
            for (int t = 0; t < 4; ++t)
              if ((ys >> t) & 1u) z ^= uint64_t(1) << idx[t];
            p.push_back({x, z});
            param.push_back(k);
          }
        }
}

static void check_rotations(int n, int n_occ, long* nw, double* cs, double* bs) {
  std::vector<PauliIn> p;
  std::vector<int32_t> param;
  uccsd_like(n, n_occ, p, param);
  const int64_t nr = int64_t(p.size());
  std::vector<double> phi(p.size()), dphi(p.size(), 1.0);
  for (double& v : phi) v = 2.0 * next_unit() - 1.0;
  struct Mode { bool reverse; int grad_mode; int b; };
  const Mode modes[3] = {{false, 0, 13}, {true, 1, 12}, {true, 2, 12}};
  for (const Mode& md : modes) {
    const std::vector<Run> runs = split_runs(p.data(), nr, md.grad_mode == 1 ? param.data() : nullptr);
    std::vector<RunData> data;
    for (const Run& r : runs) data.push_back(build_run_data(r, p.data(), phi.data(), dphi.data(), md.grad_mode));
    const std::vector<Pass> passes = schedule(runs, data, p.data(), n, md.b, 3, md.reverse, md.reverse ? 96 : 0,
                                              md.grad_mode == 1 ? 1 : 0, 1 << 16, 1 << 20);
    check_order(md.reverse ? "reverse schedule" : "forward schedule", runs, passes, p.data(), md.reverse);
    int tile_passes = 0;
    for (const Pass& ps : passes) {
      if (!ps.tile) continue;
      ++tile_passes;
      std::vector<RunRec> recs;
      std::vector<RunDesc> descs;
      for (int ri : ps.runs) descs.push_back(make_run_desc(runs[ri], data[ri], ps.qmask, 0, md.grad_mode == 2, recs));
      std::vector<uint32_t> xl;
      for (const RunDesc& d : descs) xl.push_back(uint32_t(d.x_loc));
      const int fb = popc(ps.qmask);
      for (const SegDesc& sg : segment_pass(xl, fb, 3))
        for (uint32_t j = sg.first; j < sg.first + sg.count; ++j) {
          RunDesc& d = descs[j];
          set_tile_walk(d, sg.wb_mask, fb);
          set_short_form(d, recs.data());
          // bits the run enumerates or fixes: its support (kRunEnum) or pivot (kRunFull)
          uint32_t ins = sg.wb_mask;
          if (d.mode == kRunEnum)
            for (uint32_t t = 0; t < d.n_sup; ++t) ins |= 1u << unsigned((d.sup_pack >> (8 * t)) & 0xffu);
          else if (d.mode == kRunFull)
            ins |= 1u << d.pivot;
          const uint32_t free_bits = ((1u << fb) - 1u) & ~ins;
          check_walk(md.reverse ? "reverse" : "forward", free_bits, d.walk_log, d.dep_p, d.dep_q, d.hi_mask,
                     uint32_t(d.z0_loc), d.zlane, nw, cs, bs);
        }
    }
    CHECK(tile_passes > 0, "no tile pass in mode %d", md.grad_mode);
  }
}

// Projected-sum tilings (expectation and fast lambda): a CPU walk of every
// work item of every blob, the way the tile kernels take it (lane deposit,
// register patterns, chunk words and their signs, Walsh-Hadamard transform
// over the register patterns, the subgroups' signs), must reproduce
//   sum_t c_t <psi|P_t|psi>,  <psi|P|psi> = sum_m conj(psi[m]) i^{|x&z|} (-1)^{|(m^x)&z|} psi[m^x],
// and lambda = sum_t c_t P_t psi element by element, both summed directly
// over the terms, on a seeded random state; and each batch's items must
// cover its records x chunks exactly once.  Lambda is also summed as the
// kernels sum it, in 64-bit fixed point per tile at the scale 2^s,
// s = fx_shift - e_psi (e_psi: exponent of the state's largest |re| + |im|):
// every term must stay below 2^50 (the range of the rounding by 1.5 * 2^52)
// and every slot's sum of |terms| below 2^62, and the result must match.  The sums mix random
// strings of weight <= 4, Jordan-Wigner hopping strings with number-operator
// variants (many subgroups over a Z chain) and strings whose support is too
// wide to enumerate.
static long g_x_batches = 0, g_x_multi = 0;
static double g_fx_term = 0.0;  // largest |term| * 2^s over 2^50
static double g_fx_diff = 0.0;  // largest |fixed-point lambda - H psi| / sum |c|

// One fixed-point term as the kernels form it: fma(a, b, fma(c, d, M)) with
// M = 1.5 * 2^52, read back as an integer.
static int64_t fx_term(double a, double b, double c, double d) {
  const double M = 6755399441055744.0;
  const double t = std::fma(a, b, std::fma(c, d, M));
  int64_t bits, mb;
  std::memcpy(&bits, &t, 8);
  std::memcpy(&mb, &M, 8);
  return bits - mb;
}
static double g_x_diff = 0.0;  // largest |walk - direct| / (sum |c| <psi|psi>)
static void check_expect(int n, int b, int c, int n_terms, double item_parts = 3.0) {
  const uint64_t all = (uint64_t(1) << n) - 1;
  const uint64_t low = (uint64_t(1) << c) - 1;
  std::vector<PauliIn> p;
  std::vector<double> coef;
  std::set<std::pair<uint64_t, uint64_t>> seen;
  while (int(p.size()) < n_terms) {
    const int kind = int(next_u64() % 3);
    uint64_t x = 0, z = 0;
    if (kind == 0) {
      const int w = 1 + int(next_u64() % 4);
      for (int i = 0; i < w; ++i) {
        const int q = int(next_u64() % uint64_t(n));
        const int k = int(next_u64() % 3);  // X, Y, Z
        if (k < 2) x |= uint64_t(1) << q;
        if (k > 0) z |= uint64_t(1) << q;
      }
    } else if (kind == 1) {
      int a = int(next_u64() % uint64_t(n)), d = int(next_u64() % uint64_t(n));
      if (a == d) continue;
      if (a > d) std::swap(a, d);
      x = (uint64_t(1) << a) | (uint64_t(1) << d);
      for (int q = a + 1; q < d; ++q) z |= uint64_t(1) << q;
      if (next_u64() & 1u) z |= uint64_t(1) << a;                     // X Y or Y X ends
      else z |= uint64_t(1) << d;
      if (next_u64() % 3 == 0) z ^= uint64_t(1) << (next_u64() % uint64_t(n));  // a number operator
    } else {
      const int w = kMaxSup + 1 + int(next_u64() % 2);
      for (int i = 0; i < w; ++i) x |= uint64_t(1) << (next_u64() % uint64_t(n));
      z = next_u64() & all;
    }
    x &= all;
    z &= all;
    if (!x || popc(x | low) > b || !seen.insert({x, z}).second) continue;
    p.push_back({x, z});
    coef.push_back(2.0 * next_unit() - 1.0);
  }
  std::vector<double> pr(size_t(1) << n), pi(size_t(1) << n);
  double nrm = 0.0;
  for (size_t m = 0; m < pr.size(); ++m) {
    pr[m] = 2.0 * next_unit() - 1.0;
    pi[m] = 2.0 * next_unit() - 1.0;
    nrm += pr[m] * pr[m] + pi[m] * pi[m];
  }
  // direct sum over the terms, and lambda = H psi term by term
  std::vector<double> lr_want(pr.size(), 0.0), li_want(pr.size(), 0.0);
  for (size_t t = 0; t < p.size(); ++t) {
    const int ph = popc(p[t].x & p[t].z) & 3;  // (P psi)[m] = i^ph (-1)^{|(m^x)&z|} psi[m^x]
    for (uint64_t m = 0; m <= all; ++m) {
      const uint64_t m2 = m ^ p[t].x;
      const double sg = (popc(m2 & p[t].z) & 1) ? -coef[t] : coef[t];
      const double a = sg * pr[m2], b = sg * pi[m2];
      lr_want[m] += ph == 0 ? a : ph == 1 ? -b : ph == 2 ? -a : b;
      li_want[m] += ph == 0 ? b : ph == 1 ? a : ph == 2 ? -b : -a;
    }
  }
  std::vector<double> lr_got(pr.size(), 0.0), li_got(pr.size(), 0.0);
  std::vector<double> lr_fx(pr.size(), 0.0), li_fx(pr.size(), 0.0);
  int e_psi = -4000;  // largest exponent of |re| + |im| over the state
  for (size_t m = 0; m < pr.size(); ++m) {
    const double a = std::fabs(pr[m]) + std::fabs(pi[m]);
    int e = 0;
    if (a > 0.0) {
      std::frexp(a, &e);
      e_psi = std::max(e_psi, e);
    }
  }
  double want = 0.0, scale = 0.0;
  for (size_t t = 0; t < p.size(); ++t) {
    double re = 0.0, im = 0.0;  // sum_m conj(psi[m]) (-1)^{|(m^x)&z|} psi[m^x]
    for (uint64_t m = 0; m <= all; ++m) {
      const uint64_t m2 = m ^ p[t].x;
      const double sg = (popc(m2 & p[t].z) & 1) ? -1.0 : 1.0;
      re += sg * (pr[m] * pr[m2] + pi[m] * pi[m2]);
      im += sg * (pr[m] * pi[m2] - pi[m] * pr[m2]);
    }
    const int ph = popc(p[t].x & p[t].z) & 3;  // times i^ph
    const double v = ph == 0 ? re : ph == 1 ? -im : ph == 2 ? -re : im;
    want += coef[t] * v;
    scale += std::fabs(coef[t]);
  }
  std::string err;
  const std::vector<HGroup> gs = build_groups(p.data(), coef.data(), int64_t(p.size()), &err);
  CHECK(err.empty(), "build_groups: %s", err.c_str());
  const int NW = 16;
  const HTiling T = build_tiling(gs, n, b, c, size_t(1) << 24, NW, item_parts);
  CHECK(!T.blob_overflow, "expectation blob overflow");
  CHECK(T.groups.empty(), "%zu whole-state groups", T.groups.size());
  double got = 0.0;
  long multi = 0, batches = 0;
  for (size_t tt = 0; tt < T.frames.size(); ++tt) {
    const FrameDesc& fr = T.frames[tt];
    const char* bl = reinterpret_cast<const char*>(T.blob.data() + 2 * size_t(T.blob_off[tt]));
    const XHdr* h = reinterpret_cast<const XHdr*>(bl);
    const XBatch* xb = reinterpret_cast<const XBatch*>(bl + h->off_batch);
    const XItem* items = reinterpret_cast<const XItem*>(bl + h->off_items);
    const uint32_t* start = reinterpret_cast<const uint32_t*>(bl + h->off_start);
    const XRec* recs = reinterpret_cast<const XRec*>(bl + h->off_rec);
    const TSub* subs = reinterpret_cast<const TSub*>(bl + h->off_sub);
    const double* co = reinterpret_cast<const double*>(bl + h->off_coef);
    CHECK(h->n_waves == uint32_t(NW) && start[0] == 0 && start[NW] == h->n_items, "work lists");
    batches += h->n_batches;
    // each batch's records x chunks covered once
    std::vector<std::vector<int>> cover(h->n_batches);
    for (uint32_t bi = 0; bi < h->n_batches; ++bi) {
      cover[bi].assign(size_t(xb[bi].n_rec) * xb[bi].n_chunk, 0);
      CHECK(xb[bi].n_chunk <= uint32_t(kXChunkWords) && xb[bi].n_reg <= uint32_t(kXRegBits), "batch shape");
      multi += xb[bi].n_cls > 1;
    }
    for (uint32_t i = 0; i < h->n_items; ++i) {
      const XItem& it = items[i];
      for (uint32_t r = it.recs & 0xffffu; r < (it.recs >> 16); ++r)
        for (uint32_t cc = it.chunks & 0xffffu; cc < (it.chunks >> 16); ++cc)
          cover[it.batch][size_t(r) * xb[it.batch].n_chunk + cc]++;
    }
    for (uint32_t bi = 0; bi < h->n_batches; ++bi)
      for (int v : cover[bi]) CHECK(v == 1, "batch %u: a record x chunk covered %d times", bi, v);
    const int nb = fr.b;
    uint64_t qm = 0;
    for (int j = 0; j < nb; ++j) qm |= uint64_t(1) << fr.q[j];
    const uint64_t comp = all & ~qm;
    std::vector<double> tr(size_t(1) << nb), ti(size_t(1) << nb);
    std::vector<uint64_t> glob(size_t(1) << nb);  // global index of each LDS slot
    for (uint64_t tb = 0; tb < (uint64_t(1) << popc(comp)); ++tb) {
      uint64_t base = 0;
      {
        uint64_t mm = comp;
        for (int j = 0; mm; ++j, mm &= mm - 1)
          if ((tb >> j) & 1u) base |= mm & (~mm + 1);
      }
      for (uint32_t l = 0; l < (1u << nb); ++l) {
        uint64_t g = base;
        for (int j = 0; j < nb; ++j)
          if ((l >> j) & 1u) g |= uint64_t(1) << fr.q[j];
        tr[lds_slot(l)] = pr[g];
        ti[lds_slot(l)] = pi[g];
        glob[lds_slot(l)] = g;
      }
      // the pass's fixed-point scale and the tile's accumulators
      const int sh = h->fx_shift - std::max(e_psi, -973);
      const double sc = std::ldexp(1.0, sh);
      std::vector<int64_t> ar_fx(size_t(1) << nb, 0), ai_fx(size_t(1) << nb, 0);
      std::vector<double> mag(size_t(1) << nb, 0.0);  // sum of |terms| per slot, scaled
      for (int w = 0; w < NW; ++w)
        for (uint32_t i = start[w]; i < start[w + 1]; ++i) {
          const XItem& it = items[i];
          const XBatch& B = xb[it.batch];
          const bool MULTI = B.n_cls > 1;
          const uint32_t nv = 1u << B.n_reg;
          for (uint32_t lane = 0; lane < 64; ++lane) {
            if (lane >> B.n_lane) continue;
            uint32_t dl = 0;
            for (uint32_t k = 0; k < B.n_lane; ++k) dl |= ((lane >> k) & 1u) << ((B.lane_pack >> (4 * k)) & 15u);
            const uint32_t sdl = lds_slot(dl);
            for (uint32_t r = it.recs & 0xffffu; r < (it.recs >> 16); ++r) {
              const XRec rc = recs[B.rec_off + r];
              double hr[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
              for (uint32_t cc = it.chunks & 0xffffu; cc < (it.chunks >> 16); ++cc) {
                const uint32_t u = sdl ^ rc.slot ^ (B.cword[cc] & 0x7fffffffu);
                const double sg = (B.cword[cc] >> 31) ? -1.0 : 1.0;
                for (uint32_t v = 0; v < nv; ++v) {
                  const uint32_t s2 = u ^ B.vslot[v];
                  CHECK(s2 < (1u << nb) && (s2 ^ B.sx) < (1u << nb), "slot out of the tile");
                  const double ar = tr[s2 ^ B.sx], ai = ti[s2 ^ B.sx], br = tr[s2], bi2 = ti[s2];
                  const uint32_t a = MULTI ? v : 0;
                  hr[a] += sg * (ar * br + ai * bi2);
                  hi[a] += sg * (ar * bi2 - ai * br);
                }
              }
              if (MULTI)
                for (uint32_t hh = 1; hh < nv; hh <<= 1)
                  for (uint32_t v = 0; v < nv; ++v)
                    if (!(v & hh)) {
                      const double r0 = hr[v], r1 = hr[v | hh], i0 = hi[v], i1 = hi[v | hh];
                      hr[v] = r0 + r1;
                      hr[v | hh] = r0 - r1;
                      hi[v] = i0 + i1;
                      hi[v | hh] = i0 - i1;
                    }
              uint32_t k0 = 0;
              for (uint32_t cls = 0; cls < (MULTI ? nv : 1u); ++cls) {
                const uint32_t k1 = MULTI ? B.cls_end[cls] : B.n_sub;
                for (uint32_t k = k0; k < k1; ++k) {
                  const TSub& sd = subs[B.sub_off + k];
                  const double* cv = co + 2 * (size_t(B.coef_off) + size_t(k) * B.n_rec + r);
                  const int par = popc(dl & sd.w_loc) + popc(rc.bits & sd.w_loc) + popc(base & sd.w_out);
                  const double t = cv[0] * hr[cls] - cv[1] * hi[cls];
                  got += (par & 1) ? -t : t;
                }
                k0 = k1;
              }
              if (MULTI) CHECK(k0 == B.n_sub, "classes cover %u of %u subgroups", k0, B.n_sub);
              // lambda, as the fast lambda build walks the item: G at the
              // lane's register patterns, then lam[m] += G psi[m'] and
              // lam[m'] += conj(G) psi[m] over the chunks
              double gr[4] = {0, 0, 0, 0}, gi[4] = {0, 0, 0, 0};
              uint32_t q0 = 0;
              for (uint32_t cls = 0; cls < (MULTI ? nv : 1u); ++cls) {
                const uint32_t q1 = MULTI ? B.cls_end[cls] : B.n_sub;
                for (uint32_t k = q0; k < q1; ++k) {
                  const TSub& sd = subs[B.sub_off + k];
                  const double* cv = co + 2 * (size_t(B.coef_off) + size_t(k) * B.n_rec + r);
                  const int par = popc(dl & sd.w_loc) + popc(rc.bits & sd.w_loc) + popc(base & sd.w_out);
                  gr[cls] += (par & 1) ? -cv[0] : cv[0];
                  gi[cls] += (par & 1) ? -cv[1] : cv[1];
                }
                q0 = q1;
              }
              if (MULTI)
                for (uint32_t hh = 1; hh < nv; hh <<= 1)
                  for (uint32_t v = 0; v < nv; ++v)
                    if (!(v & hh)) {
                      const double r0 = gr[v], r1 = gr[v | hh], i0 = gi[v], i1 = gi[v | hh];
                      gr[v] = r0 + r1;
                      gr[v | hh] = r0 - r1;
                      gi[v] = i0 + i1;
                      gi[v | hh] = i0 - i1;
                    }
              for (uint32_t cc = it.chunks & 0xffffu; cc < (it.chunks >> 16); ++cc) {
                const uint32_t u = sdl ^ rc.slot ^ (B.cword[cc] & 0x7fffffffu);
                const double sg = (B.cword[cc] >> 31) ? -1.0 : 1.0;
                for (uint32_t v = 0; v < nv; ++v) {
                  const uint32_t s2 = u ^ B.vslot[v], s1 = s2 ^ B.sx;  // m', m
                  const double g_r = sg * gr[MULTI ? v : 0], g_i = sg * gi[MULTI ? v : 0];
                  const uint64_t gm = glob[s1], gp = glob[s2];
                  lr_got[gm] += g_r * tr[s2] - g_i * ti[s2];  // lam[m] += G psi[m']
                  li_got[gm] += g_r * ti[s2] + g_i * tr[s2];
                  lr_got[gp] += g_r * tr[s1] + g_i * ti[s1];  // lam[m'] += conj(G) psi[m]
                  li_got[gp] += g_r * ti[s1] - g_i * tr[s1];
                  // the same in fixed point
                  const double fr_ = g_r * sc, fi_ = g_i * sc;
                  const double t1 = std::fabs(fr_) * (std::fabs(tr[s2]) + std::fabs(ti[s2]));
                  const double t2 = std::fabs(fr_) * (std::fabs(tr[s1]) + std::fabs(ti[s1]));
                  const double t3 = std::fabs(fi_) * (std::fabs(tr[s2]) + std::fabs(ti[s2]));
                  const double t4 = std::fabs(fi_) * (std::fabs(tr[s1]) + std::fabs(ti[s1]));
                  const double tm = std::max(std::max(t1, t2), std::max(t3, t4));
                  g_fx_term = std::max(g_fx_term, tm / std::ldexp(1.0, 50));
                  CHECK(tm < std::ldexp(1.0, 50), "fixed-point term %.3g reaches 2^50", tm);
                  mag[s1] += t1 + t3;
                  mag[s2] += t2 + t4;
                  ar_fx[s1] += fx_term(fr_, tr[s2], -fi_, ti[s2]);
                  ai_fx[s1] += fx_term(fr_, ti[s2], fi_, tr[s2]);
                  ar_fx[s2] += fx_term(fr_, tr[s1], fi_, ti[s1]);
                  ai_fx[s2] += fx_term(fr_, ti[s1], -fi_, tr[s1]);
                }
              }
            }
          }
        }
      for (uint32_t l = 0; l < (1u << nb); ++l) {
        CHECK(mag[l] < std::ldexp(1.0, 62), "fixed-point sum bound %.3g reaches 2^62", mag[l]);
        lr_fx[glob[l]] += std::ldexp(double(ar_fx[l]), -sh);
        li_fx[glob[l]] += std::ldexp(double(ai_fx[l]), -sh);
      }
    }
  }
  got *= 2.0;
  CHECK(std::fabs(got - want) <= 1e-12 * scale * nrm, "expectation n=%d b=%d: blob walk %.17g, direct %.17g", n, b,
        got, want);
  double lmax = 0.0;
  for (size_t m = 0; m < pr.size(); ++m)
    lmax = std::max(lmax, std::hypot(lr_got[m] - lr_want[m], li_got[m] - li_want[m]));
  CHECK(lmax <= 1e-12 * scale, "lambda n=%d b=%d: blob walk differs from H psi by %.3g", n, b, lmax);
  double fmax = 0.0;
  for (size_t m = 0; m < pr.size(); ++m)
    fmax = std::max(fmax, std::hypot(lr_fx[m] - lr_want[m], li_fx[m] - li_want[m]));
  CHECK(fmax <= 1e-12 * scale, "lambda n=%d b=%d: fixed-point walk differs from H psi by %.3g", n, b, fmax);
  g_fx_diff = std::max(g_fx_diff, fmax / scale);
  g_x_diff = std::max(g_x_diff, lmax / scale);
  CHECK(multi > 0 || n_terms < 200, "no multi-class batch (n=%d)", n);
  g_x_batches += batches;
  g_x_multi += multi;
  g_x_diff = std::max(g_x_diff, std::fabs(got - want) / (scale * nrm));
}

// Random 4-qubit rotations on 32 qubits (X/Y with an odd number of Y), in a
// 14-qubit frame with 4 fixed low qubits: three consecutive runs fill a frame
// about as far as it goes (3.07 runs per pass), so passes that reach past
// runs they commute with must hold more (about 3.8).
static void check_random_schedule() {
  const int n = 32, nr = 2000;
  std::vector<PauliIn> p;
  for (int k = 0; k < nr; ++k) {
    uint64_t x = 0, z = 0;
    int got = 0, ys = 0;
    while (got < 4) {
      const int q = int(next_u64() % uint64_t(n));
      if (x & (uint64_t(1) << q)) continue;
      x |= uint64_t(1) << q;
      if (next_u64() & 1u) { z |= uint64_t(1) << q; ++ys; }
      ++got;
    }
    if (!(ys & 1)) z ^= x & (~x + 1);  // flip the lowest factor X <-> Y: odd Y count
    p.push_back({x, z});
  }
  std::vector<double> phi(size_t(nr), 0.05);
  const std::vector<Run> runs = split_runs(p.data(), nr, nullptr);
  std::vector<RunData> data;
  for (const Run& r : runs) data.push_back(build_run_data(r, p.data(), phi.data(), nullptr, 0));
  const std::vector<Pass> passes = schedule(runs, data, p.data(), n, 14, 4, false, 0, 0, 1 << 16, 1 << 20);
  check_order("random schedule", runs, passes, p.data(), false);
  long in_tiles = 0, tiles = 0;
  for (const Pass& ps : passes)
    if (ps.tile) {
      ++tiles;
      in_tiles += long(ps.runs.size());
    }
  CHECK(tiles > 0 && double(in_tiles) / double(tiles) >= 3.5, "random schedule: %ld runs in %ld tile passes",
        in_tiles, tiles);
}

int main() {
  long nw = 0;
  double cs = 0.0, bs = 0.0;
  check_rotations(18, 6, &nw, &cs, &bs);
  check_rotations(14, 4, &nw, &cs, &bs);
  check_random_schedule();
  check_expect(12, 8, 3, 400);                             // several frames and tiles
  check_expect(9, 14, 3, 150);                             // one frame smaller than a tile
  check_expect(14, 10, 4, 600);
  check_expect(14, 10, 4, 600, 1.5);                       // the lambda tilings' coarser work items
  if (g_fail) {
    std::printf("%d failures over %ld walks\n", g_fail, nw);
    return 1;
  }
  std::printf("ok %ld walks, mean cost %.4f (least %.4f), %ld run pairs reordered; expectation: %ld batches (%ld "
              "multi-class), relative difference %.3g; fixed-point lambda: largest term %.3g of 2^50, relative "
              "difference %.3g\n",
              nw, cs / double(nw), bs / double(nw), g_moved, g_x_batches, g_x_multi, g_x_diff, g_fx_term, g_fx_diff);
  return 0;
}
