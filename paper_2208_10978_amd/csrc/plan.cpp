// Host-side planning (see plan.h).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <unordered_map>

namespace q2sv {

// ---------------------------------------------------------------------------
// runs
// ---------------------------------------------------------------------------
std::vector<Run> split_runs(const PauliIn* p, int64_t n_rot, const int32_t* param) {
  std::vector<Run> out;
  Run cur;
  for (int64_t k = 0; k < n_rot; ++k) {
    const uint64_t x = p[k].x, z = p[k].z;
    const int32_t pk = param ? param[k] : -1;
    bool join = cur.count > 0 && cur.count < kMaxRunStrings && x == cur.x && pk == cur.param;
    if (join) {
      const uint64_t d = z ^ cur.z0;
      // same-x strings commute iff |x & (z_k ^ z_0)| is even
      if (popc(x & d) & 1) join = false;
      else if (popc(cur.dmask | d) > kMaxSup) join = false;
    }
    if (join) {
      cur.dmask |= z ^ cur.z0;
      ++cur.count;
    } else {
      if (cur.count) out.push_back(cur);
      cur = Run();
      cur.first = k;
      cur.count = 1;
      cur.x = x;
      cur.z0 = z;
      cur.param = pk;
    }
  }
  if (cur.count) out.push_back(cur);
  return out;
}

static std::vector<int> bit_list(uint64_t m) {
  std::vector<int> v;
  while (m) {
    v.push_back(__builtin_ctzll(m));
    m &= m - 1;
  }
  return v;
}

RunData build_run_data(const Run& r, const PauliIn* p, const double* phi, const double* dphi, int want_grad) {
  RunData d;
  const int K = r.count;
  d.omega0 = uint32_t(popc(r.x & r.z0) & 3);
  // eps_k(m') = (omega_k / omega_0) (-1)^{|m' & (z_k ^ z_0)|}; the ratio is +/-1
  std::vector<int> neg(K), dpat(K);
  d.pat_glob = bit_list(r.dmask);
  const int L = int(d.pat_glob.size());
  for (int k = 0; k < K; ++k) {
    const uint64_t zk = p[r.first + k].z;
    const int diff = (popc(r.x & zk) - popc(r.x & r.z0)) & 3;  // 0 or 2
    neg[k] = diff == 2;
    dpat[k] = int(compress(zk ^ r.z0, r.dmask));
    if (neg[k]) d.str_neg |= uint8_t(1u << k);
    d.str_dpat[k] = uint8_t(dpat[k]);
  }
  auto entry = [&](unsigned pat, RunRec& e) {
    double ph = 0.0, a = 0.0;
    for (int k = 0; k < K; ++k) {
      const bool minus = neg[k] ^ (popc(uint64_t(pat & dpat[k])) & 1);
      ph += minus ? -phi[r.first + k] : phi[r.first + k];
      if (dphi) a += minus ? -dphi[r.first + k] : dphi[r.first + k];
    }
    e.c = std::cos(0.5 * ph);
    e.s = std::sin(0.5 * ph);
    e.a = a;
    e.eps_neg = 0;
    for (int k = 0; k < K; ++k)
      if (neg[k] ^ (popc(uint64_t(pat & dpat[k])) & 1)) e.eps_neg |= 1u << k;
  };
  d.sup_glob = bit_list(r.x);
  const int S = int(d.sup_glob.size());
  if (r.x == 0) {
    d.mode = kRunDiag;
    d.recs.resize(size_t(1) << L);
    for (unsigned pat = 0; pat < (1u << L); ++pat) entry(pat, d.recs[pat]);
    return d;
  }
  const bool enum_ok = S <= kMaxSup && (r.dmask & ~r.x) == 0;
  if (!enum_ok) {
    d.mode = kRunFull;
    d.recs.resize(size_t(1) << L);
    for (unsigned pat = 0; pat < (1u << L); ++pat) entry(pat, d.recs[pat]);
    return d;
  }
  d.mode = kRunEnum;
  const int pivot_rank = S - 1;  // the pivot is the highest support bit
  for (unsigned v = 0; v < (1u << S); ++v) {
    if (!((v >> pivot_rank) & 1u)) continue;  // m' has the pivot bit set
    uint64_t bits = 0;
    for (int j = 0; j < S; ++j) bits |= uint64_t((v >> j) & 1u) << d.sup_glob[j];
    const unsigned pat = unsigned(compress(bits, r.dmask));
    RunRec e{};
    entry(pat, e);
    e.bits = bits;
    const bool identity = (e.c == 1.0 && e.s == 0.0);
    bool keep;
    if (want_grad == 2) keep = true;
    else if (want_grad == 1) keep = !identity || e.a != 0.0;
    else keep = !identity;
    if (keep) d.recs.push_back(e);
  }
  return d;
}

FrameDesc make_frame(uint64_t qmask, int n, int c) {
  FrameDesc f{};
  int j = 0;
  for (int q = 0; q < n; ++q)
    if ((qmask >> q) & 1ull) f.q[j++] = uint8_t(q);
  f.b = uint8_t(j);
  f.c = uint8_t(c);
  int k = 0;
  for (int q = 0; q < n; ++q)
    if (!((qmask >> q) & 1ull)) {
      f.comp[k++] = uint8_t(q);
      f.comp_mask |= uint64_t(1) << q;
    }
  f.n_comp = uint8_t(k);
  return f;
}

static int local_pos(int g, uint64_t qmask) { return popc(qmask & ((uint64_t(1) << g) - 1)); }

RunDesc make_run_desc(const Run& r, const RunData& d, uint64_t qmask, uint32_t slot, int per_string,
                      std::vector<RunRec>& recs_out) {
  RunDesc rd{};
  rd.x_loc = compress(r.x, qmask);
  rd.z0_loc = compress(r.z0 & qmask, qmask);
  rd.z0_out = r.z0 & ~qmask;
  rd.omega0 = d.omega0;
  rd.slot = slot;
  rd.rec_off = uint32_t(recs_out.size());
  rd.n_rec = uint32_t(d.recs.size());
  rd.mode = d.mode;
  rd.n_str = uint32_t(r.count);
  rd.str_neg = d.str_neg;
  for (int k = 0; k < kMaxRunStrings; ++k) rd.dpat_pack |= uint64_t(d.str_dpat[k]) << (8 * k);
  rd.per_string = uint32_t(per_string);
  if (r.x) rd.pivot = uint32_t(local_pos(highest_bit(r.x), qmask));
  rd.n_sup = uint32_t(d.mode == kRunEnum ? d.sup_glob.size() : 0);
  if (d.mode == kRunEnum)
    for (size_t j = 0; j < d.sup_glob.size(); ++j)
      rd.sup_pack |= uint64_t(local_pos(d.sup_glob[j], qmask)) << (8 * j);
  rd.n_pat = uint32_t(d.mode == kRunEnum ? 0 : d.pat_glob.size());
  if (d.mode != kRunEnum)
    for (size_t j = 0; j < d.pat_glob.size(); ++j) {
      const int g = d.pat_glob[j];
      const uint64_t pos = ((qmask >> g) & 1ull) ? uint64_t(local_pos(g, qmask)) : uint64_t(64 + g);
      rd.pat_pack |= pos << (8 * j);
    }
  for (const RunRec& e : d.recs) {
    RunRec o = e;
    if (d.mode == kRunEnum) o.bits = compress(e.bits, qmask);
    recs_out.push_back(o);
  }
  return rd;
}

// Rank over GF(2) of the low `bits` bits of v[0..n).
static int low_rank(const uint32_t* v, int n, int bits) {
  uint32_t piv[32] = {};
  int r = 0;
  for (int i = 0; i < n; ++i) {
    uint32_t x = v[i] & ((1u << bits) - 1u);
    for (int k = bits - 1; k >= 0 && x; --k) {
      if (!((x >> k) & 1u)) continue;
      if (!piv[k]) {
        piv[k] = x;
        ++r;
        x = 0;
      } else {
        x ^= piv[k];
      }
    }
  }
  return r;
}

// Which free bits the lane index carries, in lane-bit order.  The LDS slots
// of 16 consecutive lanes fall on distinct banks for 8-byte words when the
// low four bits of the slots of lane bits 0..3 are independent over GF(2),
// and those of 8 lanes for 16-byte words when the low three bits of the
// slots of lane bits 0..2 are; the slot map is linear, so the first four lane
// bits are chosen to minimise the resulting conflict degrees.  The remaining
// lane bits are the lowest free bits left; bits past kWalkLaneBits go to the
// walk's loop index.
static uint32_t order_lane_bits_search(uint32_t free_bits, uint32_t (&lane_p)[kWalkLaneBits]) {
  uint32_t cand[32];
  int k = 0;
  for (uint32_t m = free_bits; m; m &= m - 1) cand[k++] = m & (~m + 1u);
  const int head = std::min(k, 4);
  int best[4] = {0, 1, 2, 3};
  double best_cost = 1e30;
  int pick[4];
  // cost of a choice: mean conflict degree of 8-byte words over 16 lanes plus
  // half that of 16-byte words over 8 lanes
  auto cost = [&](const int* ix) {
    uint32_t q[4];
    for (int i = 0; i < head; ++i) q[i] = lds_slot(cand[ix[i]]);
    const int h3 = std::min(head, 3);
    return double(1u << head) / double(1u << low_rank(q, head, 4)) +
           0.5 * double(1u << h3) / double(1u << low_rank(q, h3, 3));
  };
  std::function<bool(int)> search = [&](int d) {
    if (d == head) {
      const double c = cost(pick);
      if (c < best_cost) {
        best_cost = c;
        std::copy(pick, pick + head, best);
      }
      return best_cost <= 1.5;  // no conflicts: stop
    }
    for (int i = 0; i < k; ++i) {
      bool used = false;
      for (int j = 0; j < d; ++j) used |= pick[j] == i;
      if (used) continue;
      pick[d] = i;
      if (search(d + 1)) return true;
    }
    return false;
  };
  if (head > 0) search(0);
  int n = 0;
  uint32_t taken = 0;
  for (int i = 0; i < head; ++i) {
    lane_p[n++] = cand[best[i]];
    taken |= cand[best[i]];
  }
  for (int i = 0; i < k && n < kWalkLaneBits; ++i)
    if (!(taken & cand[i])) {
      lane_p[n++] = cand[i];
      taken |= cand[i];
    }
  for (int i = n; i < kWalkLaneBits; ++i) lane_p[i] = 0;
  return taken;
}

// The choice depends on free_bits alone; walks of one plan repeat a few
// hundred patterns, so each thread keeps the choices it has made.
static uint32_t order_lane_bits(uint32_t free_bits, uint32_t (&lane_p)[kWalkLaneBits]) {
  struct Choice {
    uint32_t lane_p[kWalkLaneBits];
    uint32_t taken;
  };
  thread_local std::unordered_map<uint32_t, Choice> memo;
  auto it = memo.find(free_bits);
  if (it == memo.end()) {
    Choice c;
    c.taken = order_lane_bits_search(free_bits, c.lane_p);
    it = memo.emplace(free_bits, c).first;
  }
  std::copy(it->second.lane_p, it->second.lane_p + kWalkLaneBits, lane_p);
  return it->second.taken;
}

void set_tile_walk(RunDesc& rd, uint32_t wb_mask, int b) {
  uint32_t ins = wb_mask;
  if (rd.mode == kRunEnum) {
    for (uint32_t j = 0; j < rd.n_sup; ++j) ins |= 1u << unsigned((rd.sup_pack >> (8 * j)) & 0xffu);
  } else if (rd.mode == kRunFull) {
    ins |= 1u << rd.pivot;
  }
  const uint32_t all = (1u << b) - 1u;
  const uint32_t free_bits = all & ~ins;
  rd.walk_log = uint32_t(popc(uint64_t(free_bits)));
  rd.zlane = 0;
  uint32_t lane_p[kWalkLaneBits];
  const uint32_t on_lanes = order_lane_bits(free_bits, lane_p);
  for (int i = 0; i < kWalkLaneBits; ++i) {
    rd.dep_p[i] = lane_p[i];
    rd.dep_q[i] = lane_p[i] ? lds_slot(lane_p[i]) : 0u;
    if (uint32_t(rd.z0_loc) & lane_p[i]) rd.zlane |= 1u << i;
  }
  rd.hi_mask = free_bits & ~on_lanes;
}

void set_short_form(RunDesc& rd, const RunRec* recs) {
  rd.sx = lds_slot(uint32_t(rd.x_loc));
  rd.short_form = rd.mode == kRunEnum && rd.n_rec <= uint32_t(kShortRecs) && rd.walk_log <= uint32_t(kWalkLaneBits);
  if (!rd.short_form) return;
  for (uint32_t r = 0; r < rd.n_rec; ++r) {
    const RunRec& e = recs[rd.rec_off + r];
    const uint32_t bits = uint32_t(e.bits);
    rd.rec_sbits[r] = lds_slot(bits);
    rd.rec_pbits[r] = uint32_t(popc(uint64_t(bits & uint32_t(rd.z0_loc))) & 1);
    rd.rec_eps[r] = e.eps_neg;
    rd.rec_c[r] = e.c;
    rd.rec_s[r] = e.s;
    rd.rec_a[r] = e.a;
  }
}

std::vector<SegDesc> segment_pass(const std::vector<uint32_t>& x_loc, int b, int region_bits) {
  std::vector<SegDesc> out;
  const uint32_t all = b >= 32 ? ~0u : ((1u << b) - 1u);
  // pick region bits outside `used`, highest first (the lanes of a wavefront
  // then walk the low, contiguous bits)
  auto pick = [&](uint32_t used) {
    uint32_t wb = 0;
    for (int p = b - 1; p >= 0 && popc(uint64_t(wb)) < region_bits; --p)
      if (!((used >> p) & 1u)) wb |= 1u << p;
    return popc(uint64_t(wb)) == region_bits ? wb : 0u;
  };
  size_t i = 0;
  while (i < x_loc.size()) {
    SegDesc sg{uint32_t(i), 0, 0, 0};
    uint32_t used = 0;
    while (i < x_loc.size()) {
      const uint32_t nu = used | (x_loc[i] & all);
      if (sg.count > 0 && popc(uint64_t(all & ~nu)) < region_bits) break;
      used = nu;
      ++sg.count;
      ++i;
      if (popc(uint64_t(all & ~used)) < region_bits) break;  // a run too wide for regions: alone
    }
    sg.wb_mask = pick(used);
    out.push_back(sg);
  }
  return out;
}

double run_line_fraction(const RunData& d, int c) {
  if (d.mode != kRunEnum) return 1.0;
  const int S = int(d.sup_glob.size());
  int low = 0;
  for (int g : d.sup_glob)
    if (g < c) ++low;
  // pairs touched: n_rec of 2^(S-1) patterns; lines hold the low support bits
  double f = double(d.recs.size()) / double(1u << (S - 1)) * double(1u << low);
  return f < 1.0 ? f : 1.0;
}

// Do two runs commute?  Their strings share one x each (x_a, x_b) and have z
// masks z0 ^ d, so by bilinearity of the symplectic form every pair of
// strings commutes iff the two reference strings do, |x_a & d| is even for
// every d of run b, and |d & x_b| is even for every d of run a.  Runs on
// disjoint qubits always commute.
bool runs_commute(const Run& a, const Run& b, const PauliIn* p) {
  if (!((a.x | a.z0 | a.dmask) & (b.x | b.z0 | b.dmask))) return true;
  if ((popc(a.x & b.z0) + popc(a.z0 & b.x)) & 1) return false;
  for (int j = 1; j < b.count; ++j)
    if (popc(a.x & (p[b.first + j].z ^ b.z0)) & 1) return false;
  for (int i = 1; i < a.count; ++i)
    if (popc((p[a.first + i].z ^ a.z0) & b.x) & 1) return false;
  return true;
}

// fill: 0 takes consecutive runs and closes the pass at the first that does
// not fit; 1 takes, among the eligible candidates, the one adding the fewest
// qubits (the earliest on ties)
static std::vector<Pass> schedule_policy(const std::vector<Run>& runs, const std::vector<RunData>& data,
                                         const PauliIn* p, int n, int b, int c, bool reverse, int max_slots_per_pass,
                                         int slots_per_run, int max_runs, int max_recs, int fill) {
  std::vector<Pass> out;
  const int R = int(runs.size());
  const uint64_t all = n >= 64 ? ~0ull : ((uint64_t(1) << n) - 1);
  if (R == 0) return out;
  if (n <= b) {
    // the whole state is one tile
    Pass ps;
    ps.tile = true;
    ps.qmask = all;
    int slots = 0, nrec = 0;
    for (int i = 0; i < R; ++i) {
      const int ri = reverse ? R - 1 - i : i;
      const int need = slots_per_run ? slots_per_run : runs[ri].count;
      const int rec = int(data[ri].recs.size());
      if ((max_slots_per_pass && slots + need > max_slots_per_pass) || int(ps.runs.size()) >= max_runs ||
          nrec + rec > max_recs) {
        out.push_back(ps);
        ps.runs.clear();
        slots = 0;
        nrec = 0;
      }
      ps.runs.push_back(ri);
      slots += need;
      nrec += rec;
    }
    out.push_back(ps);
    return out;
  }
  const uint64_t low = (uint64_t(1) << c) - 1;
  // application order: list order forward, reversed for the reverse sweep
  auto at = [&](int i) { return reverse ? R - 1 - i : i; };
  std::vector<char> taken(size_t(R), 0);
  int head = 0;
  while (head < R) {
    while (head < R && taken[size_t(at(head))]) ++head;
    if (head >= R) break;
    const int first = at(head);
    if (popc(low | runs[first].x) > b) {  // support wider than a tile: whole-state pass
      Pass ps;
      ps.tile = false;
      ps.qmask = all;
      ps.runs.push_back(first);
      out.push_back(ps);
      taken[size_t(first)] = 1;
      continue;
    }
    // Open a pass with the first run not yet scheduled.  The candidates are
    // the next kScheduleWindow unscheduled runs; a candidate may join while
    // the frame, slot and record limits allow, provided it commutes with every
    // candidate before it that is left out (the product of commuting rotations
    // does not depend on their order, and neither do the gradients
    // Im <lam|P|psi>, which are invariant under a rotation that commutes with
    // P).  Members keep list order.
    // (consecutive rule: every run from head on, as far as they fit; they are
    // all untaken, since that rule never skips one)
    std::vector<int> win;
    for (int i = head; i < R && (fill == 0 || int(win.size()) < kScheduleWindow); ++i) {
      if (taken[size_t(at(i))]) continue;
      if (fill == 0 && popc(low | runs[size_t(at(i))].x) > b) break;
      win.push_back(at(i));
      if (fill == 0 && int(win.size()) > max_runs) break;
    }
    const int W = int(win.size());
    std::vector<char> in(size_t(W), 0);
    // commutation of window candidates i < j, found when first needed
    // (0 unknown, 1 they commute, 2 they do not; the consecutive rule never
    // asks)
    std::vector<char> comm(fill == 0 ? 0 : size_t(W) * size_t(W), 0);
    auto eligible = [&](int j) {
      for (int i = 0; i < j; ++i) {
        if (in[size_t(i)]) continue;
        char& cm = comm[size_t(i) * size_t(W) + size_t(j)];
        if (!cm) cm = runs_commute(runs[size_t(win[size_t(i)])], runs[size_t(win[size_t(j)])], p) ? 1 : 2;
        if (cm == 2) return false;
      }
      return true;
    };
    uint64_t q = low;
    std::vector<int> seg;
    int slots = 0, nrec = 0;
    double alone = 0.0;
    auto join = [&](int j) {
      const int ri = win[size_t(j)];
      in[size_t(j)] = 1;
      q |= runs[size_t(ri)].x;
      slots += slots_per_run ? slots_per_run : runs[size_t(ri)].count;
      nrec += int(data[size_t(ri)].recs.size());
      seg.push_back(j);
      taken[size_t(ri)] = 1;
      alone += run_line_fraction(data[size_t(ri)], c);
    };
    join(0);  // the first unscheduled run always opens the pass
    // can window candidate j join (frame, slots, records); how many qubits
    // does it add
    auto fits = [&](int j, int* added) {
      const int ri = win[size_t(j)];
      const uint64_t nq = q | runs[size_t(ri)].x;
      *added = popc(nq) - popc(q);
      const int need = slots_per_run ? slots_per_run : runs[size_t(ri)].count;
      const int rec = int(data[size_t(ri)].recs.size());
      return popc(nq) <= b && !(max_slots_per_pass && slots + need > max_slots_per_pass) &&
             int(seg.size()) < max_runs && nrec + rec <= max_recs;
    };
    for (;;) {
      int best = -1, best_new = 65, added = 0;
      if (fill == 0) {
        const int j = int(seg.size());  // the next run in order
        if (j < W && fits(j, &added)) best = j;
      } else {
        for (int j = 1; j < W; ++j) {
          if (in[size_t(j)] || !fits(j, &added) || added >= best_new || !eligible(j)) continue;
          best = j;
          best_new = added;
          if (added == 0) break;
        }
      }
      if (best < 0) break;
      join(best);
    }
    std::sort(seg.begin(), seg.end());  // window order = application order
    for (int& j : seg) j = win[size_t(j)];
    if (seg.size() >= 2 && alone > 1.0) {
      // fill the frame up to b qubits (extra qubits only shrink the grid)
      for (int qq = 0; qq < n && popc(q) < b; ++qq) q |= uint64_t(1) << qq;
      Pass ps;
      ps.tile = true;
      ps.qmask = q;
      ps.runs = seg;
      out.push_back(ps);
    } else {
      for (int ri : seg) {
        Pass ps;
        ps.tile = false;
        ps.qmask = all;
        ps.runs.push_back(ri);
        out.push_back(ps);
      }
    }
  }
  return out;
}

std::vector<Pass> schedule(const std::vector<Run>& runs, const std::vector<RunData>& data, const PauliIn* p, int n,
                           int b, int c, bool reverse, int max_slots_per_pass, int slots_per_run, int max_runs,
                           int max_recs) {
  // both fill rules; the schedule with fewer passes wins (consecutive runs
  // suit a list ordered for locality, such as the tile-major UCCSD sequence;
  // the fewest-qubits rule packs lists of scattered rotations)
  std::vector<Pass> a = schedule_policy(runs, data, p, n, b, c, reverse, max_slots_per_pass, slots_per_run,
                                        max_runs, max_recs, 0);
  if (n <= b) return a;
  size_t in_tiles = 0, tiles = 0;
  for (const Pass& ps : a)
    if (ps.tile) {
      ++tiles;
      in_tiles += ps.runs.size();
    }
  if (tiles && in_tiles >= 8 * tiles) return a;  // consecutive runs already share passes well
  std::vector<Pass> f = schedule_policy(runs, data, p, n, b, c, reverse, max_slots_per_pass, slots_per_run,
                                        max_runs, max_recs, 1);
  return f.size() < a.size() ? f : a;
}

// ---------------------------------------------------------------------------
// grouped Pauli sums
// ---------------------------------------------------------------------------
std::vector<HGroup> build_groups(const PauliIn* p, const double* coef, int64_t n_terms, std::string* err) {
  std::map<uint64_t, std::vector<int64_t>> by_x;
  for (int64_t t = 0; t < n_terms; ++t) by_x[p[t].x].push_back(t);
  std::vector<HGroup> out;
  out.reserve(by_x.size());
  for (auto& kv : by_x) {
    HGroup g;
    g.x = kv.first;
    g.diag = g.x == 0;
    g.sup = bit_list(g.x);
    const int S = int(g.sup.size());
    g.enumerated = !g.diag && S <= kMaxSup;
    const uint64_t smask = g.enumerated ? g.x : 0;
    // subgroups by w = z outside the enumerated support
    std::map<uint64_t, std::vector<int64_t>> by_w;
    for (int64_t t : kv.second) by_w[p[t].z & ~smask].push_back(t);
    std::vector<uint64_t> recs;
    if (g.enumerated) {
      for (unsigned v = 0; v < (1u << S); ++v) {
        if (!((v >> (S - 1)) & 1u)) continue;
        uint64_t bits = 0;
        for (int j = 0; j < S; ++j) bits |= uint64_t((v >> j) & 1u) << g.sup[j];
        recs.push_back(bits);
      }
    } else {
      recs.push_back(0);
    }
    const int NR = int(recs.size());
    std::vector<uint64_t> ws;
    std::vector<double> re, im;
    double tmax = 0.0;
    for (auto& wv : by_w) {
      ws.push_back(wv.first);
      for (int r = 0; r < NR; ++r) {
        // T_w[r] = sum_t c_t i^{|x & z_t|} (-1)^{|m' & z_t^S|}
        double a = 0.0, b = 0.0;
        for (int64_t t : wv.second) {
          const int ph = popc(g.x & p[t].z) & 3;
          const int sg = popc(recs[r] & p[t].z & smask) & 1;
          double cr = 0.0, ci = 0.0;
          const double cv = sg ? -coef[t] : coef[t];
          switch (ph) {
            case 0: cr = cv; break;
            case 1: ci = cv; break;
            case 2: cr = -cv; break;
            default: ci = -cv; break;
          }
          a += cr;
          b += ci;
        }
        re.push_back(a);
        im.push_back(b);
        tmax = std::max(tmax, std::hypot(a, b));
      }
    }
    // drop records whose entries vanish in every subgroup (exact zeros up to
    // the rounding of the term sums: below 1e-14 of the largest entry)
    const double tol = 1e-14 * tmax;
    std::vector<int> keep;
    for (int r = 0; r < NR; ++r) {
      bool nz = !g.enumerated;
      for (size_t w = 0; w < ws.size() && !nz; ++w)
        if (std::hypot(re[w * NR + r], im[w * NR + r]) > tol) nz = true;
      if (nz) keep.push_back(r);
    }
    if (keep.empty()) continue;  // the group is zero
    g.w = ws;
    for (int r : keep) g.rec_v.push_back(recs[r]);
    if (!g.enumerated) g.rec_v.clear();
    for (size_t w = 0; w < ws.size(); ++w)
      for (int r : keep) {
        g.t_re.push_back(re[w * NR + r]);
        g.t_im.push_back(im[w * NR + r]);
      }
    out.push_back(std::move(g));
  }
  (void)err;
  return out;
}

static GroupDesc make_group_desc(const HGroup& g, uint64_t qmask, uint32_t sub_off, uint32_t rec_off) {
  GroupDesc d{};
  d.x_loc = compress(g.x, qmask);
  d.n_sub = uint32_t(g.w.size());
  d.sub_off = sub_off;
  d.rec_off = rec_off;
  d.n_rec = uint16_t(g.n_rec());
  d.enumerated = g.enumerated;
  d.is_diag = g.diag;
  d.n_sup = uint8_t(g.enumerated ? g.sup.size() : 0);
  if (g.x) d.pivot = uint8_t(local_pos(highest_bit(g.x), qmask));
  if (g.enumerated)
    for (size_t j = 0; j < g.sup.size(); ++j) d.sup_pack |= uint64_t(local_pos(g.sup[j], qmask)) << (8 * j);
  return d;
}

// whole-state group (identity frame) with its own coefficient array
static void append_full_group(HTiling& t, const HGroup& g, uint64_t all) {
  const uint32_t sub_off = uint32_t(t.subs.size());
  const uint32_t rec_off = uint32_t(t.recbits.size());
  t.groups.push_back(make_group_desc(g, all, sub_off, rec_off));
  const int NR = g.n_rec();
  for (size_t w = 0; w < g.w.size(); ++w) {
    SubDesc s{};
    s.w_loc = g.w[w];
    s.w_out = 0;
    s.coef_off = uint32_t(t.coef.size() / 2);
    for (int r = 0; r < NR; ++r) {
      t.coef.push_back(g.t_re[w * NR + r]);
      t.coef.push_back(g.t_im[w * NR + r]);
    }
    t.subs.push_back(s);
  }
  for (uint64_t v : g.rec_v) t.recbits.push_back(v);
}

// A group's share of a blob (its records, subgroups, coefficients and a
// batch), for cutting a tile's groups into blobs of bounded size.
static size_t group_blob_bytes(const HGroup& g) {
  const size_t nr = size_t(g.n_rec());
  return sizeof(XBatch) + sizeof(XItem) + nr * sizeof(XRec) + g.w.size() * (sizeof(TSub) + nr * 16);
}

// ---------------------------------------------------------------------------
// projected-sum blobs of the expectation and lambda (see XBatch)
// ---------------------------------------------------------------------------
namespace {

// Bits of v spread over the set bits of mask, ascending.
uint32_t deposit_bits(uint32_t v, uint32_t mask) {
  uint32_t out = 0;
  for (int j = 0; mask; ++j, mask &= mask - 1)
    if ((v >> j) & 1u) out |= mask & (~mask + 1u);
  return out;
}

// The lane / register / chunk split of one batch's free bits.
struct XSplit {
  uint32_t lane[kXLaneBits] = {};  // single-bit masks, lane-bit order
  int n_lane = 0;
  uint32_t lane_mask = 0, reg_mask = 0, chunk_mask = 0;
};

// Free bits F of a group: the first four lane bits are the bank-conflict-free
// choice for F; the deviation bits D (where the batch's subgroups differ
// from w0) go to the remaining lane bits and then to the register bits, which
// are padded with bits that no subgroup mask touches where possible (a
// register bit of a subgroup would give it a nonzero class).  Returns false
// when D does not fit.
bool x_split(uint32_t F, uint32_t D, uint32_t W, XSplit& out) {
  const int nf = popc(uint64_t(F));
  uint32_t lp[kWalkLaneBits];
  order_lane_bits(F, lp);
  out = XSplit{};
  out.n_lane = std::min(kXLaneBits, nf);
  const int head = std::min(4, out.n_lane);
  uint32_t used = 0;
  for (int i = 0; i < head; ++i) {
    out.lane[i] = lp[i];
    used |= lp[i];
  }
  // remaining lane bits: deviation bits first, then the lowest free bits
  int li = head;
  for (uint32_t m = D & F & ~used; m && li < out.n_lane; m &= m - 1, ++li) {
    out.lane[li] = m & (~m + 1u);
    used |= out.lane[li];
  }
  for (uint32_t m = F & ~used; m && li < out.n_lane; m &= m - 1, ++li) {
    out.lane[li] = m & (~m + 1u);
    used |= out.lane[li];
  }
  out.lane_mask = used;
  const int n_reg = std::min(kXRegBits, nf - out.n_lane);
  uint32_t reg = 0;
  int ri = 0;
  for (uint32_t m = D & F & ~used; m; m &= m - 1) {
    if (ri == n_reg) return false;
    reg |= m & (~m + 1u);
    ++ri;
  }
  for (uint32_t m = F & ~used & ~reg & ~W; m && ri < n_reg; m &= m - 1, ++ri) reg |= m & (~m + 1u);
  for (uint32_t m = F & ~used & ~reg; m && ri < n_reg; m &= m - 1, ++ri) reg |= m & (~m + 1u);
  out.reg_mask = reg;
  out.chunk_mask = F & ~used & ~reg;
  return true;
}

// Bitwise majority of masks (ties: 0).
uint32_t majority(const std::vector<uint32_t>& v, const std::vector<int>& idx) {
  uint32_t out = 0;
  for (int bit = 0; bit < 32; ++bit) {
    int ones = 0;
    for (int k : idx) ones += int((v[size_t(k)] >> bit) & 1u);
    if (2 * ones > int(idx.size())) out |= 1u << bit;
  }
  return out;
}

uint32_t deviation(const std::vector<uint32_t>& v, const std::vector<int>& idx, uint32_t w0) {
  uint32_t d = 0;
  for (int k : idx) d |= v[size_t(k)] ^ w0;
  return d;
}

}  // namespace

void pack_expect_blob(HTiling& t, const std::vector<HGroup>& gs, const std::vector<int>& members, uint64_t qmask,
                      size_t max_blob, int n_waves, double item_parts) {
  const int fb = popc(qmask);
  const uint32_t all = fb >= 32 ? ~0u : ((1u << fb) - 1u);
  std::vector<XBatch> xb;
  std::vector<double> cost;
  std::vector<XRec> xr;
  std::vector<TSub> ts;
  std::vector<double> co;
  double g_max = 0.0, g_sum = 0.0;  // bounds on |G| (largest, and summed over groups)
  for (int gi : members) {
    const HGroup& g = gs[size_t(gi)];
    const uint32_t x_loc = uint32_t(compress(g.x, qmask));
    const uint32_t smask = g.enumerated ? x_loc : (1u << local_pos(highest_bit(g.x), qmask));
    const uint32_t F = all & ~smask;
    const int NR = g.n_rec();
    const uint32_t rec_off = uint32_t(xr.size());
    for (int r = 0; r < NR; ++r) {
      XRec rc{};
      rc.bits = g.enumerated ? uint32_t(compress(g.rec_v[size_t(r)], qmask)) : smask;
      rc.slot = lds_slot(rc.bits);
      xr.push_back(rc);
    }
    const int K = int(g.w.size());
    std::vector<uint32_t> wl(static_cast<size_t>(K)), wf(static_cast<size_t>(K));
    uint32_t W = 0;
    for (int k = 0; k < K; ++k) {
      wl[size_t(k)] = uint32_t(compress(g.w[size_t(k)] & qmask, qmask));
      wf[size_t(k)] = wl[size_t(k)] & F;
      W |= wf[size_t(k)];
    }
    // batches: every subgroup at once with w0 = 0 (no chunk signs) when
    // their free bits fit, else with the majority mask when the deviation
    // fits, else greedy from the first remaining subgroup
    std::vector<std::pair<std::vector<int>, uint32_t>> batches;
    std::vector<int> rest(static_cast<size_t>(K));
    for (int k = 0; k < K; ++k) rest[size_t(k)] = k;
    XSplit sp;
    if (x_split(F, W, W, sp)) {
      batches.emplace_back(rest, 0u);
      rest.clear();
    }
    while (!rest.empty()) {
      uint32_t w0 = majority(wf, rest);
      if (x_split(F, deviation(wf, rest, w0), W, sp)) {
        batches.emplace_back(rest, w0);
        break;
      }
      w0 = wf[size_t(rest[0])];
      std::vector<int> take{rest[0]}, left;
      uint32_t D = 0;
      for (size_t i = 1; i < rest.size(); ++i) {
        const uint32_t d2 = D | (wf[size_t(rest[i])] ^ w0);
        if (x_split(F, d2, W, sp)) {
          take.push_back(rest[i]);
          D = d2;
        } else {
          left.push_back(rest[i]);
        }
      }
      const uint32_t wm = majority(wf, take);
      const uint32_t dm = deviation(wf, take, wm);
      if (popc(uint64_t(dm)) < popc(uint64_t(D)) && x_split(F, dm, W, sp)) w0 = wm;
      batches.emplace_back(take, w0);
      rest.swap(left);
    }
    // |re| + |im| of T_k[r] summed over the group's subgroups: a bound on
    // |G| at the pairs of record r; a slot meets one record of the group
    std::vector<double> rec_abs(static_cast<size_t>(NR), 0.0);
    for (auto& bt : batches) {
      const std::vector<int>& mem = bt.first;
      const uint32_t w0 = bt.second;
      const bool ok = x_split(F, deviation(wf, mem, w0), W, sp);
      if (!ok) t.blob_overflow = true;  // a one-subgroup batch always fits
      XBatch b{};
      for (int i = 0; i < kXLaneBits; ++i)
        if (i < sp.n_lane) b.lane_pack |= uint32_t(__builtin_ctz(sp.lane[i])) << (4 * i);
      b.n_lane = uint32_t(sp.n_lane);
      b.n_reg = uint32_t(popc(uint64_t(sp.reg_mask)));
      b.n_chunk = 1u << popc(uint64_t(sp.chunk_mask));
      if (b.n_chunk > uint32_t(kXChunkWords)) t.blob_overflow = true;
      b.sx = lds_slot(x_loc);
      b.n_rec = uint32_t(NR);
      b.rec_off = rec_off;
      for (uint32_t v = 0; v < (1u << kXRegBits); ++v)
        b.vslot[v] = v < (1u << b.n_reg) ? lds_slot(deposit_bits(v, sp.reg_mask)) : 0u;
      for (uint32_t cc = 0; cc < b.n_chunk && cc < uint32_t(kXChunkWords); ++cc) {
        const uint32_t u = deposit_bits(cc, sp.chunk_mask);
        b.cword[cc] = lds_slot(u) | (uint32_t(popc(uint64_t(u & w0)) & 1) << 31);
        b.signed_chunks |= b.cword[cc] >> 31;
      }
      // subgroups sorted by class (their register bits, in v coordinates)
      std::vector<std::pair<uint32_t, int>> by_cls;
      for (int k : mem) by_cls.emplace_back(uint32_t(compress(wl[size_t(k)], sp.reg_mask)), k);
      std::stable_sort(by_cls.begin(), by_cls.end(),
                       [](const std::pair<uint32_t, int>& a, const std::pair<uint32_t, int>& c2) { return a.first < c2.first; });
      b.n_sub = uint32_t(mem.size());
      b.sub_off = uint32_t(ts.size());
      b.coef_off = uint32_t(co.size() / 2);
      uint32_t seen = 0;
      for (size_t i = 0; i < by_cls.size(); ++i) {
        const int k = by_cls[i].second;
        seen |= 1u << by_cls[i].first;
        TSub sd{};
        sd.w_loc = wl[size_t(k)];
        sd.w_out = g.w[size_t(k)] & ~qmask;
        ts.push_back(sd);
        for (int r = 0; r < NR; ++r) {
          co.push_back(g.t_re[size_t(k) * size_t(NR) + size_t(r)]);
          co.push_back(g.t_im[size_t(k) * size_t(NR) + size_t(r)]);
          rec_abs[size_t(r)] += std::fabs(co[co.size() - 2]) + std::fabs(co.back());
        }
      }
      for (uint32_t v = 0; v < (1u << kXRegBits); ++v) {
        uint32_t end = 0;
        for (const auto& e : by_cls)
          if (e.first <= v) ++end;
        b.cls_end[v] = end;
      }
      b.n_cls = seen == 1u ? 1u : uint32_t(popc(uint64_t(seen))) + 1u;  // 1: class 0 alone
      xb.push_back(b);
      const double pos = double(NR) * double(uint64_t(1) << popc(uint64_t(F))) / 64.0;
      cost.push_back(pos * 11.0 + double(NR) * (40.0 + 8.0 * double(mem.size()) + (b.n_cls > 1 ? 16.0 : 0.0)));
    }
    double worst = 0.0;
    for (double a : rec_abs) worst = std::max(worst, a);
    g_max = std::max(g_max, worst);
    g_sum += worst;
  }
  // work items: batches cut (by records, then by chunks) to at most
  // 1/item_parts of a wavefront's share, then longest first onto the least
  // loaded wavefront
  const int NW = std::max(1, n_waves);
  double total = 0.0;
  for (double v : cost) total += v;
  const double target = std::max(1.0, total / double(NW) / std::max(item_parts, 0.25));
  std::vector<XItem> items;
  std::vector<double> icost;
  for (size_t bi = 0; bi < xb.size(); ++bi) {
    const XBatch& b = xb[bi];
    const uint32_t parts = uint32_t(std::min(1024.0, std::ceil(cost[bi] / target)));
    auto add = [&](uint32_t r0, uint32_t r1, uint32_t c0, uint32_t c1) {
      XItem it{};
      it.batch = uint32_t(bi);
      it.recs = r0 | r1 << 16;
      it.chunks = c0 | c1 << 16;
      items.push_back(it);
      icost.push_back(cost[bi] * double(r1 - r0) * double(c1 - c0) / (double(b.n_rec) * double(b.n_chunk)));
    };
    if (parts <= b.n_rec) {
      for (uint32_t p = 0; p < parts; ++p) add(b.n_rec * p / parts, b.n_rec * (p + 1) / parts, 0, b.n_chunk);
    } else {
      const uint32_t cp = std::min(b.n_chunk, (parts + b.n_rec - 1) / b.n_rec);
      for (uint32_t r = 0; r < b.n_rec; ++r)
        for (uint32_t p = 0; p < cp; ++p) add(r, r + 1, b.n_chunk * p / cp, b.n_chunk * (p + 1) / cp);
    }
  }
  std::vector<int> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = int(i);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c2) { return icost[size_t(a)] > icost[size_t(c2)]; });
  std::vector<double> load(size_t(NW), 0.0);
  std::vector<std::vector<int>> lists(static_cast<size_t>(NW));
  for (int i : order) {
    const size_t w = size_t(std::min_element(load.begin(), load.end()) - load.begin());
    load[w] += icost[size_t(i)];
    lists[w].push_back(i);
  }
  std::vector<XItem> list;
  std::vector<uint32_t> start;
  for (auto& l : lists) {
    std::sort(l.begin(), l.end());
    start.push_back(uint32_t(list.size()));
    for (int i : l) list.push_back(items[size_t(i)]);
  }
  start.push_back(uint32_t(list.size()));
  auto align16 = [](size_t v) { return (v + 15) & ~size_t(15); };
  XHdr h{};
  {
    // binary exponents with g_max < 2^e_g and g_sum < 2^e_s (frexp; 0 for 0)
    int e_g = 0, e_s = 0;
    std::frexp(g_max, &e_g);
    std::frexp(g_sum * (1.0 + 1e-12), &e_s);
    h.fx_shift = std::min(50 - e_g, 62 - e_s);
  }
  h.n_batches = uint32_t(xb.size());
  h.n_items = uint32_t(list.size());
  h.n_waves = uint32_t(NW);
  size_t off = sizeof(XHdr);
  h.off_batch = uint32_t(align16(off));
  off = h.off_batch + xb.size() * sizeof(XBatch);
  h.off_items = uint32_t(align16(off));
  off = h.off_items + list.size() * sizeof(XItem);
  h.off_start = uint32_t(align16(off));
  off = h.off_start + start.size() * sizeof(uint32_t);
  h.off_rec = uint32_t(align16(off));
  off = h.off_rec + xr.size() * sizeof(XRec);
  h.off_sub = uint32_t(align16(off));
  off = h.off_sub + ts.size() * sizeof(TSub);
  h.off_coef = uint32_t(align16(off));
  off = h.off_coef + co.size() * sizeof(double);
  h.bytes = uint32_t(align16(off));
  if (h.bytes > max_blob) t.blob_overflow = true;
  std::vector<unsigned char> bytes(h.bytes, 0);
  std::memcpy(bytes.data(), &h, sizeof(h));
  auto put = [&](uint32_t at, const void* src, size_t n) {
    if (n) std::memcpy(bytes.data() + at, src, n);
  };
  put(h.off_batch, xb.data(), xb.size() * sizeof(XBatch));
  put(h.off_items, list.data(), list.size() * sizeof(XItem));
  put(h.off_start, start.data(), start.size() * sizeof(uint32_t));
  put(h.off_rec, xr.data(), xr.size() * sizeof(XRec));
  put(h.off_sub, ts.data(), ts.size() * sizeof(TSub));
  put(h.off_coef, co.data(), co.size() * sizeof(double));
  t.blob_off.push_back(uint32_t(t.blob.size() / 2));
  const size_t at = t.blob.size();
  t.blob.resize(at + h.bytes / 8);
  std::memcpy(t.blob.data() + at, bytes.data(), h.bytes);
}

HTiling build_tiling(const std::vector<HGroup>& gs, int n, int b, int c, size_t max_blob, int n_waves,
                     double item_parts) {
  HTiling t;
  t.b = b;
  t.c = c;
  const uint64_t all = n >= 64 ? ~0ull : ((uint64_t(1) << n) - 1);
  const uint64_t low = (uint64_t(1) << c) - 1;
  const int G = int(gs.size());
  std::vector<int> tile_of(G, -1);
  std::vector<uint64_t> tile_q;
  const size_t fixed = sizeof(XHdr) + 64;
  if (n <= b) {
    tile_q.push_back(all);
    for (int g = 0; g < G; ++g)
      if (!gs[g].diag) tile_of[g] = 0;
  } else {
    std::vector<int> todo;
    for (int g = 0; g < G; ++g)
      if (!gs[g].diag && popc(gs[g].x | low) <= b && group_blob_bytes(gs[g]) + fixed <= max_blob)
        todo.push_back(g);
    while (!todo.empty()) {
      // seed with the widest uncovered support, then add the qubit that
      // completes most uncovered groups (ties: most partial progress)
      int seed = todo[0];
      for (int g : todo)
        if (popc(gs[g].x & ~low) > popc(gs[seed].x & ~low)) seed = g;
      uint64_t q = low | gs[seed].x;
      while (popc(q) < b) {
        std::vector<double> score(n, 0.0);
        for (int g : todo) {
          const uint64_t miss = gs[g].x & ~q;
          const int k = popc(miss);
          if (k == 0) continue;
          const double v = k == 1 ? 1e6 : 1.0 / k;
          for (uint64_t mm = miss; mm; mm &= mm - 1) score[__builtin_ctzll(mm)] += v;
        }
        int best = -1;
        for (int qq = 0; qq < n; ++qq)
          if (!((q >> qq) & 1ull) && (best < 0 || score[qq] > score[best])) best = qq;
        q |= uint64_t(1) << best;
      }
      const int tid = int(tile_q.size());
      tile_q.push_back(q);
      std::vector<int> rest;
      for (int g : todo) {
        if ((gs[g].x & ~q) == 0) tile_of[g] = tid;
        else rest.push_back(g);
      }
      todo.swap(rest);
    }
    // The cover fills its first frames with every group they happen to
    // contain, which leaves those passes bound by their pair arithmetic and
    // the last ones by HBM.  Reassign each group, largest first, to the
    // least loaded frame that contains its support (load: the pairs its
    // records enumerate, a little more per subgroup).
    std::vector<int> order;
    for (int g = 0; g < G; ++g)
      if (tile_of[g] >= 0) order.push_back(g);
    auto cost = [&](int g) {
      const HGroup& h = gs[g];
      const int s = h.enumerated ? popc(h.x) : 1;
      return double(h.n_rec()) * std::ldexp(1.0, b - s) * (1.0 + 0.1 * double(h.w.size()));
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c2) { return cost(a) > cost(c2); });
    std::vector<double> load(tile_q.size(), 0.0);
    for (int g : order) {
      int best = -1;
      for (size_t tt = 0; tt < tile_q.size(); ++tt)
        if ((gs[g].x & ~tile_q[tt]) == 0 && (best < 0 || load[tt] < load[size_t(best)])) best = int(tt);
      tile_of[g] = best;
      load[size_t(best)] += cost(g);
    }
    if (tile_q.empty()) {
      uint64_t q = low;
      for (int qq = c; qq < n && popc(q) < b; ++qq) q |= uint64_t(1) << qq;
      tile_q.push_back(q);
    }
  }
  t.n_tiles = int(tile_q.size());
  for (int tt = 0; tt < t.n_tiles; ++tt) {
    const uint64_t q = tile_q[tt];
    std::vector<int> members;
    for (int g = 0; g < G; ++g)
      if (tile_of[g] == tt) members.push_back(g);
    // chunks of at most max_blob bytes
    std::vector<int> chunk;
    size_t bytes = fixed;
    auto flush = [&]() {
      t.frames.push_back(make_frame(q, n, c));
      pack_expect_blob(t, gs, chunk, q, max_blob, n_waves, item_parts);
      chunk.clear();
      bytes = fixed;
    };
    for (int g : members) {
      const size_t gb = group_blob_bytes(gs[g]) + 16;
      if (!chunk.empty() && bytes + gb > max_blob) flush();
      chunk.push_back(g);
      bytes += gb;
    }
    if (!chunk.empty() || tt == 0) flush();
  }
  for (int g = 0; g < G; ++g)
    if (tile_of[g] < 0 && !gs[g].diag) append_full_group(t, gs[g], all);
  return t;
}

}  // namespace q2sv
