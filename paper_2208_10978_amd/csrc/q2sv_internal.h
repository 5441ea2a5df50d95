// Internal descriptors shared by the host planner and the gfx950 kernels.
//
// Vocabulary.
//   frame   A pass works on blocks of 2^B amplitudes.  The block's qubits are
//           a sorted set Q (frame-local bit j is global qubit Q[j]); the other
//           n - B qubits are fixed per block and form its base index.  Q
//           always holds the lowest c qubits, so a row of 2^c amplitudes is
//           contiguous in memory.  The identity frame (B = n, base 0) is the
//           whole state.
//   run     Consecutive strings of a rotation list with one x mask that
//           commute.  On each amplitude pair (m, m ^ x) every string of the
//           run acts as +/- the same 2x2 operator, so the run is one rotation
//           by an angle Phi that depends on m only through a few "pattern"
//           bits (Section 5.1, Eq. 11: the strings of one UCC excitation form
//           such a run).
//   group   All terms of a Pauli sum that share one x mask (Section 3.1,
//           Eq. 1-2): one read of the pair (psi[m], psi[m ^ x]) serves every
//           z-variant.
//   record  An "active" value of the partner index m' = m ^ x on the support
//           of x: the pair is processed only when the run (or group) does not
//           act as the identity (or zero) there.  Pairs are enumerated per
//           record, so skipped patterns cost nothing.
#pragma once

#include <cstdint>

namespace q2sv {

constexpr int kMaxSup = 6;          // support bits enumerated per run / group
constexpr int kMaxRunStrings = 8;   // strings fused into one run
constexpr int kMaxFrameBits = 14;   // largest LDS tile (2^14 complex64)

enum RunMode : uint8_t {
  kRunEnum = 0,   // pattern bits inside the support; enumerate active records
  kRunFull = 1,   // every pair; per-pair pattern lookup into a 2^L table
  kRunDiag = 2,   // x == 0: a phase on every amplitude; 2^L table
};

// One run of commuting same-x rotations, in the coordinates of its frame.
// Every field is a full 32 or 64 bits, so tile kernels reading descriptors
// from global memory with a uniform index get scalar loads.
constexpr int kWalkLaneBits = 6;    // walk positions carried by the lane index

// LDS slot of frame-local index l.  A tile walk's lanes differ in the free
// bits of a run or group, which are often all above bit 3; unswizzled, their
// 16-byte elements would then share LDS banks.  XORing the low four bits with
// a fold of the higher ones spreads them.  The map is linear over GF(2)
// (slot(a ^ b) = slot(a) ^ slot(b)), keeps bits 4 and up, and is a bijection
// on [0, 2^B) for every B.  (constexpr: usable by host planning and kernels.)
constexpr uint32_t lds_slot(uint32_t l) { return l ^ (((l >> 4) ^ (l >> 5) ^ (l >> 7) ^ (l >> 10)) & 15u); }
struct alignas(16) RunDesc {
  // Short-form head (kRunEnum, at most kShortRecs records, walk_log <= 6: one
  // position per lane): every uniform field a tile walk needs, contiguous so
  // a kernel fetches it in one batch of scalar loads; the records inline,
  // with the LDS slot and the z0 parity of their bits on S'.
  uint32_t short_form;
  uint32_t n_rec;      // number of records, or 2^L table entries
  uint32_t omega0;     // reference phase i^{|x & z0|}, as a power of i
  uint32_t walk_log;   // tile walk: 2^walk_log positions per record
  uint32_t zlane;      // lane bit i -> z0 bit at dep_p[i]
  uint32_t sx;         // LDS slot of x_loc
  uint32_t slot;       // first gradient slot of the run
  uint32_t pad0;
  uint64_t z0_loc;     // reference string's z, frame-local bits
  uint64_t z0_out;     // reference string's z, global bits outside the frame
  // Tile walk: position t = lane + 64 j of the bits the run leaves free
  // (not enumerated, not region bits).  Lane bit i lands on frame-local bit
  // dep_p[i] (0 past the walk's width), whose LDS slot is dep_q[i]; the bits
  // of j land on the free bits hi_mask above them.
  uint32_t dep_q[kWalkLaneBits];
  uint32_t rec_sbits[2];           // slot(bits)
  uint32_t rec_pbits[2];           // parity(bits & z0_loc)
  uint32_t pad1[2];
  double rec_c[2], rec_s[2], rec_a[2];
  // rest
  uint64_t x_loc;      // flip mask (frame-local bits)
  uint32_t rec_off;    // first record (kRunEnum) or table entry (kRunFull/Diag)
  uint32_t mode;       // RunMode
  uint32_t n_str;      // strings fused in the run
  uint32_t str_neg;    // bit k: omega_k / omega_0 = -1            (kRunFull/Diag)
  uint32_t n_sup;      // support bits (kRunEnum)
  uint32_t pivot;      // frame-local highest bit of x             (kRunFull)
  uint32_t n_pat;      // pattern bits L                           (kRunFull/Diag)
  uint32_t per_string; // gradient slots are per string (else one per run)
  uint32_t hi_mask;
  uint32_t rec_eps[2];             // eps_neg
  // Position lists packed one byte per entry (entry j in bits 8j..8j+7), so
  // kernels read them with shifts instead of indexing a private array:
  uint64_t sup_pack;   // frame-local support positions, ascending
  uint64_t pat_pack;   // pattern bit j: frame-local position, or 64 + global
                       // position when outside the frame
  uint64_t dpat_pack;  // per string: pattern mask of z_k ^ z0
  uint32_t dep_p[kWalkLaneBits];
};
constexpr int kShortRecs = 2;

// A segment of a tile pass: consecutive runs none of whose x masks touches
// the frame-local bits wb_mask.  Wavefront w owns the amplitudes whose
// wb_mask bits spell w and applies the segment's runs to them with no block
// barrier (pairs never leave a region); with wb_mask = 0 wavefront 0 owns the
// whole tile.
struct alignas(16) SegDesc {
  uint32_t first;      // first run (index into the pass's descriptors)
  uint32_t count;
  uint32_t wb_mask;
  uint32_t pad;
};

// A record (kRunEnum) or table entry (kRunFull/Diag) of a run:
//   c, s  cos(Phi/2), sin(Phi/2) of the fused rotation on this pattern
//   a     sum_k dphi_k/dtheta * eps_k (parameter-gradient weight)
//   bits  frame-local bits of m' on the support (kRunEnum only)
//   eps_neg  bit k: eps_k = -1 on this pattern (kRunEnum only)
struct alignas(16) RunRec {
  uint64_t bits;
  uint32_t eps_neg;
  uint32_t pad0;
  double c;
  double s;
  double a;
  double pad1;
};

// One group of a Pauli sum in frame coordinates:
//   G(m) = sum_w (-1)^{|m' & w|} T_w[r],   m' = m ^ x,
// where r is the active record of m' (its support bits) when the group is
// enumerated, and 0 otherwise.  (H_x psi)[m] = G(m) psi[m'].
struct alignas(16) GroupDesc {
  uint64_t x_loc;      // flip mask (frame-local)
  uint32_t n_sub;      // w subgroups
  uint32_t sub_off;    // first subgroup
  uint32_t rec_off;    // first record: bits of m' on the support
  uint16_t n_rec;      // records (1 when not enumerated)
  uint8_t enumerated;  // support bits enumerated (records are patterns)
  uint8_t is_diag;     // x == 0
  uint8_t n_sup;       // support bits (enumerated groups)
  uint8_t pivot;       // frame-local highest bit of x (non-enumerated groups)
  uint16_t pad0;
  uint64_t sup_pack;   // support positions, one byte each, ascending
};

// w of one subgroup; its values T_w[r] for every record r of the group sit at
// coef[coef_off + r] (complex: re, im).
struct alignas(16) SubDesc {
  uint64_t w_loc;
  uint64_t w_out;
  uint32_t coef_off;
  uint32_t pad0;
  uint64_t pad1;
};

// ---------------------------------------------------------------------------
// Group tables of one Hamiltonian tile pass (read in place through scalar
// loads).  Every non-diagonal group is treated as pairs (m, m' = m ^ x) with
// the pivot (highest) bit of m clear.  "Enumerated bits" S' are the support
// of x (when it has at most kMaxSup bits) or the pivot alone; a record fixes
// the bits of m' on S', and each record gives two outputs: m' (coefficient
// conj(G)) and m (coefficient G), where
//   G(m) = sum_w (-1)^{|m' & w|} T_w[record]   and  (H_x psi)[m] = G(m) psi[m'].
// Each subgroup w is a TSub; the blob layout is XHdr (below).
// ---------------------------------------------------------------------------
struct alignas(16) TSub {
  uint64_t w_out;      // w, global bits outside the frame
  uint32_t w_loc;      // w, frame-local bits
  uint32_t pad;
};

// ---------------------------------------------------------------------------
// Tile passes of the expectation and of lambda (projected sums).  For one group and record r the
// pairs' contribution is Re sum_k T_k[r] S_k with
//   S_k = sum_{m'} (-1)^{|m' & w_k|} conj(psi[m' ^ x]) psi[m'].
// The free bits F of the group (frame bits outside S') are split into
//   L  six lane bits (the lane index, deposited),
//   R  up to kXRegBits register bits (a position block v held in registers;
//      two: with eight the accumulators and loads of complex64 spill),
//   C  chunk bits (the loop index),
// with every w_k agreeing with one reference mask w0 on C.  A lane then sums
// P = conj(psi[m]) psi[m'] over its chunks, signed by (-1)^{|m' & w0|}, into
// one accumulator per v; at the end of the record the Walsh-Hadamard
// transform over v gives each subgroup's sum from the entry of its R bits,
// and the lane, record and out-of-frame bits of w_k give its sign.  Per pair
// the work no longer grows with the number of subgroups.  A group whose
// subgroups differ on more free bits than L and R hold is split into batches
// (each batch one pass over the pairs).
// ---------------------------------------------------------------------------
constexpr int kXLaneBits = 6;
constexpr int kXRegBits = 2;
constexpr int kXChunkWords = 32;   // 2^|C| at most (|F| <= 13 in a 14-bit frame)

struct alignas(16) XHdr {
  uint32_t n_batches;
  uint32_t n_waves;    // wavefronts the work lists were balanced for
  uint32_t off_batch;  // byte offsets from the start of the blob
  uint32_t off_items;  // XItem work items in wavefront order: wave w takes [start[w], start[w + 1])
  uint32_t off_start;  // n_waves + 1 list starts
  uint32_t off_rec;    // XRec per record
  uint32_t off_sub;    // TSub per subgroup, each batch's sorted by class
  uint32_t off_coef;   // T_k[r] (re, im) at coef_off + k * n_rec + r
  uint32_t bytes;
  uint32_t n_items;
  // lambda builds: the fixed-point sums use the scale 2^(fx_shift - e_psi),
  // e_psi the binary exponent of psi's largest |re| + |im|
  // (fx_shift = min(50 - e_g, 62 - e_s), with every record's bound on |G|
  // below 2^e_g and the sum of those bounds below 2^e_s)
  int32_t fx_shift;
  uint32_t pad;
};

struct alignas(16) XBatch {
  uint32_t lane_pack;  // frame-local position of lane bit i in bits 4i..4i+3
  uint32_t n_lane;     // lane bits (6 unless the frame is small)
  uint32_t n_reg;      // register bits
  uint32_t n_chunk;    // 2^|C|
  uint32_t sx;         // LDS slot of x_loc
  uint32_t n_cls;      // classes present: 1 means every subgroup has class 0
  uint32_t n_rec, rec_off;
  uint32_t n_sub, sub_off, coef_off;
  uint32_t signed_chunks;  // some chunk word carries a sign (w0 meets C)
  uint32_t cls_end[1 << kXRegBits];  // subgroups of class v: [cls_end[v - 1], cls_end[v]) (from 0)
  uint32_t vslot[1 << kXRegBits];    // LDS slot of register pattern v
  uint32_t cword[kXChunkWords];  // chunk c: LDS slot of its bits | parity(bits & w0) << 31
};

// A work item: records [r0, r1) and chunks [c0, c1) of one batch (a large
// batch is split so that the wavefronts' lists balance).
struct alignas(16) XItem {
  uint32_t batch;
  uint32_t recs;       // r0 | r1 << 16
  uint32_t chunks;     // c0 | c1 << 16
  uint32_t pad;
};

struct alignas(8) XRec {
  uint32_t bits;       // frame-local bits of m' on S'
  uint32_t slot;       // their LDS slot
};

// Frame of a tile pass.
struct alignas(16) FrameDesc {
  uint8_t q[kMaxFrameBits];   // global position of frame-local bit j (q[j] = j for j < c)
  uint8_t b;                  // B
  uint8_t c;                  // contiguous low qubits
  uint8_t comp[48];           // global positions of the other qubits, ascending
  uint8_t n_comp;             // n - B
  uint8_t pad[7];
  uint64_t comp_mask;         // the same positions as a mask
};

}  // namespace q2sv
