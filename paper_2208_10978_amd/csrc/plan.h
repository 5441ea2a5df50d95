// Host-side planning: fused runs of a rotation list, their per-pattern
// tables, LDS tile schedules, and the grouped form of a Pauli sum.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "q2sv_internal.h"

namespace q2sv {

struct PauliIn { uint64_t x, z; };

inline int popc(uint64_t v) { return __builtin_popcountll(v); }
inline int highest_bit(uint64_t v) { return 63 - __builtin_clzll(v); }

// bits of v at the positions of mask, packed in ascending order
inline uint64_t compress(uint64_t v, uint64_t mask) {
  uint64_t out = 0;
  int j = 0;
  while (mask) {
    const int p = __builtin_ctzll(mask);
    out |= ((v >> p) & 1ull) << j;
    ++j;
    mask &= mask - 1;
  }
  return out;
}

// ---------------------------------------------------------------------------
// rotation runs
// ---------------------------------------------------------------------------
struct Run {
  int64_t first = 0;   // index of the first rotation
  int count = 0;       // strings in the run
  uint64_t x = 0;      // common flip mask
  uint64_t z0 = 0;     // reference z (first string)
  uint64_t dmask = 0;  // union of z_k ^ z0: the pattern bits
  int32_t param = -1;  // common parameter (parameter mode), else -1
};

// Split a rotation list into runs: consecutive strings with one x mask that
// commute with the run's first string, at most kMaxRunStrings strings and
// kMaxSup pattern bits; in parameter mode a run also has one parameter.
std::vector<Run> split_runs(const PauliIn* p, int64_t n_rot, const int32_t* param);

// Host image of one run's data for one call (angles known).
struct RunData {
  uint8_t mode = kRunFull;
  std::vector<RunRec> recs;   // records (kRunEnum) or table (kRunFull/Diag)
  uint8_t str_neg = 0;
  uint8_t str_dpat[kMaxRunStrings] = {};
  std::vector<int> pat_glob;  // pattern bit positions (global), ascending
  std::vector<int> sup_glob;  // support positions (global), ascending
  uint32_t omega0 = 0;
};

// Tables of a run.  want_grad: 0 forward only, 1 parameter gradient (needs A),
// 2 per-string gradient (every pair contributes).
RunData build_run_data(const Run& r, const PauliIn* p, const double* phi, const double* dphi, int want_grad);

// Descriptor of a run in a frame (frame qubits qmask; identity frame when
// qmask covers all n qubits).  Records are appended to `recs_out`.
RunDesc make_run_desc(const Run& r, const RunData& d, uint64_t qmask, uint32_t slot, int per_string,
                      std::vector<RunRec>& recs_out);

FrameDesc make_frame(uint64_t qmask, int n, int c);

// Fill a tile descriptor's walk for a segment with region bits wb_mask in a
// frame of b bits.
void set_tile_walk(RunDesc& rd, uint32_t wb_mask, int b);

// After set_tile_walk: inline the records of a short run (recs indexed by the
// descriptor's rec_off).
void set_short_form(RunDesc& rd, const RunRec* recs);

// Split a tile pass (its runs' frame-local x masks, in application order)
// into segments that leave region_bits frame bits untouched; region bits are
// chosen per segment.  A run whose x leaves fewer free bits forms a segment
// of its own with wb_mask = 0.
std::vector<SegDesc> segment_pass(const std::vector<uint32_t>& x_loc, int b, int region_bits);

// Fraction of the state's bytes a kRunEnum run moves when applied alone
// (lines of 2^c amplitudes are moved whole).
double run_line_fraction(const RunData& d, int c);

struct Pass {
  bool tile = false;
  uint64_t qmask = 0;
  std::vector<int> runs;   // in application order
};

// Whether every string of run a commutes with every string of run b (p: the
// rotation list the runs index).
bool runs_commute(const Run& a, const Run& b, const PauliIn* p);

// Greedy schedule.  forward: runs in list order; reverse: runs in reverse
// order.  Each pass opens with the first unscheduled run and takes later runs
// (within kScheduleWindow unscheduled runs) whose qubits still fit the frame,
// as long as each commutes with every run it passes over (at most
// kScheduleSkip of them).  A pass becomes an LDS tile pass when it holds at
// least two runs and is cheaper than applying its runs one by one.  A tile
// pass holds at most max_runs runs and max_recs records.
constexpr int kScheduleWindow = 64;
constexpr int kScheduleSkip = 16;
std::vector<Pass> schedule(const std::vector<Run>& runs, const std::vector<RunData>& data, const PauliIn* p, int n,
                           int b, int c, bool reverse, int max_slots_per_pass, int slots_per_run, int max_runs,
                           int max_recs);

// ---------------------------------------------------------------------------
// grouped Pauli sums
// ---------------------------------------------------------------------------
struct HGroup {
  uint64_t x = 0;
  bool diag = false;
  bool enumerated = false;
  std::vector<int> sup;            // support positions (global), ascending
  std::vector<uint64_t> rec_v;     // enumerated: global bits of m' on the support
  std::vector<uint64_t> w;         // subgroup masks
  std::vector<double> t_re, t_im;  // [sub * n_rec + rec]
  int n_rec() const { return int(rec_v.empty() ? 1 : rec_v.size()); }
};

std::vector<HGroup> build_groups(const PauliIn* p, const double* coef, int64_t n_terms, std::string* err);

// Device-ready arrays of one tiling of a grouped sum.  Every non-diagonal
// group whose support fits (with the c low qubits) in b qubits belongs to one
// tile; a tile's groups are packed into one or more blobs (passes) of at most
// max_blob bytes; the remaining groups run over the whole state.

struct HTiling {
  int b = 0, c = 0;
  std::vector<FrameDesc> frames;         // per pass
  std::vector<uint32_t> blob_off;        // per pass, in 16-byte words
  std::vector<uint64_t> blob;            // concatenated blobs (2 words per 16 bytes)
  std::vector<GroupDesc> groups;         // whole-state groups
  std::vector<SubDesc> subs;
  std::vector<uint64_t> recbits;
  std::vector<double> coef;              // whole-state group coefficients (re, im)
  int n_tiles = 0;
  bool blob_overflow = false;            // a blob exceeded max_blob (never expected)
};

// Frames (greedy cover of the groups' flip masks, then each group moved to
// the least loaded frame that contains it) and one projected-sum blob (XHdr)
// per frame and at most max_blob bytes, with per-wavefront work lists
// balanced for n_waves wavefronts from work items of at most 1/item_parts of
// a wavefront's share (finer items balance better but repeat each record's
// set-up); groups that fit no b-bit frame become whole-state groups.
HTiling build_tiling(const std::vector<HGroup>& gs, int n, int b, int c, size_t max_blob, int n_waves,
                     double item_parts = 3.0);

// One projected-sum blob (XHdr) of a tile's groups, appended to t.
void pack_expect_blob(HTiling& t, const std::vector<HGroup>& gs, const std::vector<int>& members, uint64_t qmask,
                      size_t max_blob, int n_waves, double item_parts = 3.0);

}  // namespace q2sv
