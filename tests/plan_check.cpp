// Host checks of the tile-walk planning (CPU only, built with the host
// compiler against plan.cpp).  For seeded Jordan-Wigner-shaped rotation lists
// (forward, per-parameter and per-string reverse schedules) and a seeded
// Pauli sum (lambda tilings with region segments, and the expectation
// tiling), the segments of a lambda tile must cover its groups in order with
// flip masks that avoid their region bits (and general groups must insert
// zeros at their support and region bits), and every walk must
//   * split the bits its run leaves free (not enumerated, not region bits)
//     into at most six lane bits and the loop bits hi_mask, disjointly;
//   * visit each of the 2^walk_log free-bit patterns exactly once;
//   * carry the LDS slot of each lane bit and its z (or w) parity bit;
//   * use lane bits whose bank-conflict cost (largest number of lanes on one
//     bank word: 16 lanes for 8-byte words, 8 lanes for 16-byte words, the
//     latter weighted by one half) is the least over every ordered choice of
//     free bits for lane bits 0..3.
// Prints "ok ..." and exits 0, or names the first failure and exits 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
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

static void check_lambda(int n, int b, long* nw, double* cs, double* bs, int rb) {
  // one- and two-body shaped terms: x on 0, 2 or 4 orbitals, Z chains, odd Y
  std::vector<PauliIn> p;
  std::vector<double> coef;
  for (int t = 0; t < 6000; ++t) {
    const int kind = int(next_u64() % 3);
    uint64_t x = 0, z = 0;
    if (kind == 0) {
      z = next_u64() & next_u64() & ((uint64_t(1) << n) - 1);
    } else {
      const int nx = kind == 1 ? 2 : 4;
      int idx[4];
      for (int i = 0; i < nx;) {
        const int q = int(next_u64() % uint64_t(n));
        if (x & (uint64_t(1) << q)) continue;
        x |= uint64_t(1) << q;
        idx[i++] = q;
      }
      std::sort(idx, idx + nx);
      for (int pr = 0; pr < nx; pr += 2)
        for (int q = idx[pr] + 1; q < idx[pr + 1]; ++q) z |= uint64_t(1) << q;
      uint32_t ys = 0;
      while (!(__builtin_popcount(ys) & 1)) ys = uint32_t(next_u64() % (1u << nx));
      for (int i = 0; i < nx; ++i)
        if ((ys >> i) & 1u) z ^= uint64_t(1) << idx[i];
    }
    p.push_back({x, z});
    coef.push_back(2.0 * next_unit() - 1.0);
  }
  std::string err;
  const std::vector<HGroup> gs = build_groups(p.data(), coef.data(), int64_t(p.size()), &err);
  CHECK(err.empty(), "build_groups: %s", err.c_str());
  std::vector<HGroup> nd;
  for (const HGroup& g : gs)
    if (!g.diag) nd.push_back(g);
  const HTiling T = build_tiling(nd, n, b, 3, true, size_t(1) << 24, rb);
  long n_fast = 0, n_seg = 0;
  for (size_t t = 0; t < T.frames.size(); ++t) {
    const char* blob = reinterpret_cast<const char*>(T.blob.data() + 2 * size_t(T.blob_off[t]));
    const TileHdr* h = reinterpret_cast<const TileHdr*>(blob);
    const TFast* fs = reinterpret_cast<const TFast*>(blob + h->off_fast);
    const TGroup* tg = reinterpret_cast<const TGroup*>(blob + sizeof(TileHdr));
    const LamSeg* sg = reinterpret_cast<const LamSeg*>(blob + h->off_segs);
    // segments cover the groups and fast records in order; every member's
    // flip mask avoids the segment's region bits
    uint32_t g_next = 0, f_next = 0;
    for (uint32_t si = 0; si < h->n_segs; ++si, ++n_seg) {
      const LamSeg& S = sg[si];
      const int nb = __builtin_popcount(S.wb_mask);
      CHECK(nb == 0 || nb == kLambdaRegionBits, "segment region mask %x", S.wb_mask);
      CHECK(S.wb_mask < (1u << b), "segment region mask %x outside the frame", S.wb_mask);
      CHECK(S.g_first == g_next && S.f_first == f_next, "segments out of order");
      CHECK(nb > 0 || S.g_count + S.f_count == 1, "a maskless segment holds %u groups", S.g_count + S.f_count);
      g_next += S.g_count;
      f_next += S.f_count;
      for (uint32_t i = S.g_first; i < S.g_first + S.g_count; ++i) {
        CHECK(!(tg[i].x_loc & S.wb_mask), "group x %x touches region bits %x", tg[i].x_loc, S.wb_mask);
        // zero insertions: S' and the region bits, ascending
        uint32_t want = tg[i].sup_mask | S.wb_mask, got = 0, prev = 0;
        for (uint32_t j = 0; j < tg[i].n_sins; ++j) {
          const uint32_t pos = uint32_t(tg[i].sins_pack >> (4 * j)) & 15u;
          CHECK(j == 0 || pos > prev, "insertions not ascending");
          prev = pos;
          got |= 1u << pos;
        }
        CHECK(got == want, "insertions %x, want %x", got, want);
      }
      for (uint32_t i = S.f_first; i < S.f_first + S.f_count; ++i, ++n_fast) {
        const TFast& f = fs[i];
        CHECK(!(f.x_loc & S.wb_mask), "fast x %x touches region bits %x", f.x_loc, S.wb_mask);
        const uint32_t free_bits = ((1u << b) - 1u) & ~f.sup_mask & ~S.wb_mask;
        check_walk("lambda", free_bits, f.walk_log, f.dep_p, f.dep_q, f.hi_mask, f.w_loc, f.wlane, nw, cs, bs);
      }
    }
    if (rb == 0) {
      // expectation tilings: no segments; walks over the bits outside S'
      CHECK(h->n_segs == 0, "segments in an expectation tiling");
      for (uint32_t i = 0; i < h->n_fast; ++i, ++n_fast) {
        const TFast& f = fs[i];
        const uint32_t free_bits = ((1u << b) - 1u) & ~f.sup_mask;
        check_walk("expect", free_bits, f.walk_log, f.dep_p, f.dep_q, f.hi_mask, f.w_loc, f.wlane, nw, cs, bs);
      }
      continue;
    }
    CHECK(g_next == h->n_groups && f_next == h->n_fast, "segments cover %u/%u groups, %u/%u fast records", g_next,
          h->n_groups, f_next, h->n_fast);
  }
  CHECK(n_fast > 0, "no fast records");
  CHECK(rb == 0 || n_seg > 0, "no segments");
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
  check_lambda(18, 12, &nw, &cs, &bs, kLambdaRegionBits);  // lambda, complex build
  check_lambda(18, 13, &nw, &cs, &bs, kLambdaRegionBits);  // lambda, real-part tiles
  check_lambda(18, 13, &nw, &cs, &bs, 0);                  // expectation (complex128 frames)
  if (g_fail) {
    std::printf("%d failures over %ld walks\n", g_fail, nw);
    return 1;
  }
  std::printf("ok %ld walks, mean cost %.4f (least %.4f), %ld run pairs reordered\n", nw, cs / double(nw),
              bs / double(nw), g_moved);
  return 0;
}
