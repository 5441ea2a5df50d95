// C ABI of libq2sv.so (declared in include/q2sv.h): argument checks, plan
// caches, staging of per-call tables, and the order of kernel launches for
// each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/q2sv.h"
#include "launch.h"
#include "plan.h"

using namespace q2sv;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Sticky device failure.  The first failed HIP call on a device marks it, and
// every later call that would use that device returns SV_EDEVICE with the
// first message: after a launch or runtime failure the device's state (and
// any work queued on it) can no longer be trusted.  t_dev is the device of
// the call in progress on this host thread.
constexpr int kMaxDevices = 64;
struct DeviceHealth {
  std::atomic<int> bad{0};
  std::mutex mu;
  std::string first;
};
DeviceHealth g_health[kMaxDevices];
thread_local int t_dev = 0;

DeviceHealth& health(int dev) { return g_health[(dev >= 0 && dev < kMaxDevices) ? dev : 0]; }

int device_fail(const std::string& msg) {
  DeviceHealth& h = health(t_dev);
  {
    std::lock_guard<std::mutex> lk(h.mu);
    if (!h.bad.load()) h.first = msg;
    h.bad.store(1);
  }
  return fail(SV_EDEVICE, msg);
}

// SV_OK, or SV_EDEVICE when the device has failed before
int device_check(int dev) {
  DeviceHealth& h = health(dev);
  if (!h.bad.load()) return SV_OK;
  std::lock_guard<std::mutex> lk(h.mu);
  return fail(SV_EDEVICE, "device " + std::to_string(dev) + " is unusable after an earlier failure: " + h.first);
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return device_fail(std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

uint64_t fnv(const void* data, size_t bytes, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < bytes; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

// Device buffer that grows; growing waits for the stream that uses it.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  int ensure(size_t bytes, hipStream_t st) {
    if (bytes <= cap) return SV_OK;
    if (p) {
      if (hipStreamSynchronize(st) != hipSuccess) return device_fail("hipStreamSynchronize failed");
      hipFree(p);
      p = nullptr;
      cap = 0;
    }
    size_t want = std::max<size_t>(bytes, 4096);
    want = std::max(want, cap * 2);
    if (hipMalloc(&p, want) != hipSuccess) {
      p = nullptr;
      return fail(SV_ENOMEM, "device scratch allocation of " + std::to_string(want) + " bytes failed");
    }
    cap = want;
    return SV_OK;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

// Pinned staging buffer; reuse waits until the previous upload has left it.
struct Staging {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
  int ensure(size_t bytes) {
    if (!done && hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess)
      return device_fail("hipEventCreate failed");
    if (pending) {
      if (hipEventSynchronize(done) != hipSuccess) return device_fail("hipEventSynchronize failed");
      pending = false;
    }
    if (bytes <= cap) return SV_OK;
    if (host) hipHostFree(host);
    host = nullptr;
    size_t want = std::max<size_t>(bytes, 1 << 16);
    want = std::max(want, cap * 2);
    if (hipHostMalloc(&host, want, hipHostMallocDefault) != hipSuccess) {
      host = nullptr;
      cap = 0;
      return fail(SV_ENOMEM, "pinned staging allocation failed");
    }
    cap = want;
    return SV_OK;
  }
  void release() {
    if (done) {
      hipEventSynchronize(done);
      hipEventDestroy(done);
    }
    if (host) hipHostFree(host);
    host = nullptr;
    done = nullptr;
    cap = 0;
  }
};

// Packs several host arrays into one upload.
struct Packer {
  std::vector<std::pair<const void*, size_t>> parts;
  std::vector<size_t> offs;
  size_t total = 0;
  size_t add(const void* p, size_t bytes) {
    total = (total + 255) & ~size_t(255);
    const size_t off = total;
    parts.push_back({p, bytes});
    offs.push_back(off);
    total += bytes;
    return off;
  }
};

int upload(Staging& stg, DevBuf& dev, Packer& pk, hipStream_t st) {
  if (pk.total == 0) return SV_OK;
  int rc = stg.ensure(pk.total);
  if (rc) return rc;
  rc = dev.ensure(pk.total, st);
  if (rc) return rc;
  for (size_t i = 0; i < pk.parts.size(); ++i)
    if (pk.parts[i].second) std::memcpy(static_cast<char*>(stg.host) + pk.offs[i], pk.parts[i].first, pk.parts[i].second);
  HIP_TRY(hipMemcpyAsync(dev.p, stg.host, pk.total, hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(stg.done, st));
  stg.pending = true;
  return SV_OK;
}

template <typename T>
const T* dptr(const DevBuf& d, size_t off) {
  return reinterpret_cast<const T*>(static_cast<const char*>(d.p) + off);
}

int full_grid(uint64_t work) {
  const uint64_t want = (work + 255) / 256;
  return int(std::min<uint64_t>(std::max<uint64_t>(want, 1), kPartialStride));
}

// ---------------------------------------------------------------------------
// opt-in kernel timing: a HIP event pair per launch on its stream
// ---------------------------------------------------------------------------
enum ProfClass {
  kPFill, kPRunFull, kPTileFwd, kPTileRev, kPTileHExp, kPTileHLam, kPGroupFull, kPDot, kPSmall, kPCount
};
const char* kProfName[kPCount] = {"k_fill_basis", "k_run_full", "k_tile_forward", "k_tile_reverse",
                                  "k_tile_hamiltonian_expect", "k_tile_hamiltonian_lambda", "k_group_full",
                                  "k_dot", "small"};

struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double bytes;
};

struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
  }
};
Profiler g_prof;

struct ProfScope {
  hipStream_t st;
  int cls;
  double bytes;
  hipEvent_t a = nullptr;
  ProfScope(hipStream_t s, int c, double b) : st(s), cls(c), bytes(b) {
    if (!g_prof.on) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    a = g_prof.get();
    hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    hipEvent_t b = g_prof.get();
    hipEventRecord(b, st);
    g_prof.recs.push_back({cls, a, b, bytes});
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// resident Pauli sums
// ---------------------------------------------------------------------------
struct DevTiling {
  HTiling host;
  DevBuf buf;
  size_t o_frames = 0, o_boff = 0, o_blob = 0, o_groups = 0, o_subs = 0, o_recs = 0, o_coef = 0;
};

struct sv_hamiltonian {
  int n = 0;
  int64_t n_terms = 0;
  uint64_t key = 0;
  std::vector<sv_pauli> src_p;       // the term list of a per-state cached sum (compared on reuse)
  std::vector<double> src_c;
  std::vector<HGroup> groups;        // non-diagonal groups
  bool real = true;                  // every group coefficient is real (then a real psi gives a real lambda)
  std::vector<uint64_t> diag_z;      // diagonal (x = 0) terms
  std::vector<double> diag_c;
  // [dtype][role]: 0 expectation; lambda 1 complex, 2 real-part tiles
  static constexpr int kRoles = 3;
  DevTiling tilings[3][kRoles];
  bool built[3][kRoles] = {};
  DevBuf diag_dev;                   // resident diagonal d[m], FP64, 2^n entries
  bool diag_built = false;
  hipEvent_t diag_ready = nullptr;   // recorded after the diagonal's build
  int device = 0;
  std::mutex mu;                     // the lazy builds (tilings, diagonal) of a shared handle
};

static int num_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  }
  return cus;
}

static int tiling_get(sv_hamiltonian* h, int dtype, int role, DevTiling** out) {
  std::lock_guard<std::mutex> lk(h->mu);
  DevTiling& t = h->tilings[dtype][role];
  if (!h->built[dtype][role]) {
    const int b = role == 0 ? tile_bits_one(dtype) : role == 1 ? tile_bits_lambda(dtype) : kTileLamReal;
    const int c = std::min(row_bits(dtype), h->n);
    // kernels read the tables through scalar loads, so a tile's groups need
    // not be split
    // work items: a third of a wavefront's share for the expectation, two
    // thirds for lambda (whose per-record set-up weighs more than its pair
    // imbalance: 28-qubit real lambda 392 -> 378 ms)
    t.host = build_tiling(h->groups, h->n, b, c, size_t(1) << 24, role == 0 ? kExpectThreads / 64 : kLambdaThreads / 64,
                          role == 0 ? 3.0 : 1.5);
    if (t.host.blob_overflow) return fail(SV_EINVAL, "internal: a tile's group tables are too large");
    Packer pk;
    t.o_frames = pk.add(t.host.frames.data(), t.host.frames.size() * sizeof(FrameDesc));
    t.o_boff = pk.add(t.host.blob_off.data(), t.host.blob_off.size() * sizeof(uint32_t));
    t.o_blob = pk.add(t.host.blob.data(), t.host.blob.size() * sizeof(uint64_t));
    t.o_groups = pk.add(t.host.groups.data(), t.host.groups.size() * sizeof(GroupDesc));
    t.o_subs = pk.add(t.host.subs.data(), t.host.subs.size() * sizeof(SubDesc));
    t.o_recs = pk.add(t.host.recbits.data(), t.host.recbits.size() * sizeof(uint64_t));
    t.o_coef = pk.add(t.host.coef.data(), t.host.coef.size() * sizeof(double));
    std::vector<char> blob(pk.total + 1);
    for (size_t i = 0; i < pk.parts.size(); ++i)
      if (pk.parts[i].second) std::memcpy(blob.data() + pk.offs[i], pk.parts[i].first, pk.parts[i].second);
    int rc = t.buf.ensure(pk.total + 256, nullptr);
    if (rc) return rc;
    HIP_TRY(hipMemcpy(t.buf.p, blob.data(), pk.total, hipMemcpyHostToDevice));
    h->built[dtype][role] = true;
  }
  *out = &t;
  return SV_OK;
}

// The diagonal part of H as a resident FP64 vector, built once on the first
// caller's stream (8 bytes per amplitude); later callers on other streams
// wait for that build through an event.
static int diag_get(sv_hamiltonian* h, hipStream_t st, const double** out) {
  if (h->diag_z.empty()) {
    *out = nullptr;
    return SV_OK;
  }
  std::lock_guard<std::mutex> lk(h->mu);
  if (!h->diag_built) {
    const uint64_t n_amp = uint64_t(1) << h->n;
    const size_t tb = h->diag_z.size() * (sizeof(uint64_t) + sizeof(double));
    int rc = h->diag_dev.ensure(n_amp * sizeof(double) + tb + 256, st);
    if (rc) return rc;
    char* base = static_cast<char*>(h->diag_dev.p);
    uint64_t* dz = reinterpret_cast<uint64_t*>(base + n_amp * sizeof(double));
    double* dc = reinterpret_cast<double*>(dz + h->diag_z.size());
    HIP_TRY(hipMemcpy(dz, h->diag_z.data(), h->diag_z.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dc, h->diag_c.data(), h->diag_c.size() * sizeof(double), hipMemcpyHostToDevice));
    ProfScope prof(st, kPSmall, double(n_amp) * 8.0);
    HIP_TRY(launch_diag_build(reinterpret_cast<double*>(base), n_amp, dz, dc, int(h->diag_z.size()), st));
    if (!h->diag_ready) HIP_TRY(hipEventCreateWithFlags(&h->diag_ready, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(h->diag_ready, st));
    h->diag_built = true;
  }
  // a caller on another stream waits for the build (a no-op on the building stream)
  HIP_TRY(hipStreamWaitEvent(st, h->diag_ready, 0));
  *out = static_cast<const double*>(h->diag_dev.p);
  return SV_OK;
}

static int validate_paulis(const sv_pauli* p, int64_t n, int nq, const char* what) {
  if (n < 0) return fail(SV_EINVAL, std::string(what) + ": negative count");
  if (n > 0 && !p) return fail(SV_EINVAL, std::string(what) + ": NULL array");
  const uint64_t lim = nq >= 64 ? ~0ull : ((uint64_t(1) << nq) - 1);
  for (int64_t k = 0; k < n; ++k)
    if ((p[k].x | p[k].z) & ~lim)
      return fail(SV_EINVAL, std::string(what) + "[" + std::to_string(k) + "] acts on a qubit >= n");
  return SV_OK;
}

// A real state (SV_R64) stays real only under real rotations: R(P, phi) is a
// real matrix exactly when P = i^{|x&z|} X^x Z^z is imaginary, i.e. when
// |x & z| (the number of Y factors) is odd.
static int validate_real_rotations(const sv_state* s, const sv_pauli* p, int64_t n);

static int validate_finite(const double* v, int64_t n, const char* what) {
  if (n > 0 && !v) return fail(SV_EINVAL, std::string(what) + ": NULL array");
  for (int64_t k = 0; k < n; ++k)
    if (!std::isfinite(v[k])) return fail(SV_EINVAL, std::string(what) + "[" + std::to_string(k) + "] is not finite");
  return SV_OK;
}

static int hamiltonian_make(int n, const sv_pauli* p, const double* coef, int64_t n_terms, sv_hamiltonian** out) {
  int rc = validate_paulis(p, n_terms, n, "pauli sum");
  if (rc) return rc;
  rc = validate_finite(coef, n_terms, "coef");
  if (rc) return rc;
  std::unique_ptr<sv_hamiltonian> h(new sv_hamiltonian());
  h->n = n;
  h->n_terms = n_terms;
  std::string err;
  std::vector<HGroup> all = build_groups(reinterpret_cast<const PauliIn*>(p), coef, n_terms, &err);
  for (HGroup& g : all) {
    if (g.diag) {
      for (size_t w = 0; w < g.w.size(); ++w) {
        h->diag_z.push_back(g.w[w]);
        h->diag_c.push_back(g.t_re[w]);
      }
    } else {
      for (double v : g.t_im) h->real &= v == 0.0;
      h->groups.push_back(std::move(g));
    }
  }
  hipGetDevice(&h->device);
  *out = h.release();
  return SV_OK;
}

static void hamiltonian_destroy(sv_hamiltonian* h) {
  if (!h) return;
  for (auto& row : h->tilings)
    for (auto& t : row) t.buf.release();
  h->diag_dev.release();
  if (h->diag_ready) hipEventDestroy(h->diag_ready);
  delete h;
}

// ---------------------------------------------------------------------------
// state
// ---------------------------------------------------------------------------
struct sv_state {
  int n = 0;
  int dtype = SV_C128;
  void* amps = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  DevBuf scratch;      // reduction partials
  DevBuf tables;       // per-call uploaded tables
  DevBuf small;        // a few FP64 values
  Staging staging;
  double* host_word = nullptr;  // pinned FP64 word for a device value the host must read
  sv_hamiltonian* cached_h = nullptr;  // last Pauli sum passed as raw arrays
  bool real_hint = false;              // the caller asserts psi is real on entry to the adjoint calls
  std::atomic<int> busy{0};            // a call on this handle is in progress
  uint64_t amp_count() const { return uint64_t(1) << n; }
  double bytes() const { return double(amp_count()) * double(amp_bytes(dtype)); }
};

static int validate_real_rotations(const sv_state* s, const sv_pauli* p, int64_t n) {
  if (s->dtype != SV_R64) return SV_OK;
  for (int64_t k = 0; k < n; ++k)
    if (!(__builtin_popcountll(p[k].x & p[k].z) & 1))
      return fail(SV_EINVAL, "rotation[" + std::to_string(k) +
                                 "] is not real (its string has an even number of Y factors); a real state takes "
                                 "only real rotations");
  return SV_OK;
}

// The adjoint calls on a real state need lambda = H psi real: every group
// coefficient of the sum real.
static int validate_real_sum(const sv_state* s, const sv_hamiltonian* h) {
  if (s->dtype != SV_R64 || h->real) return SV_OK;
  return fail(SV_EINVAL, "a real state's adjoint needs a Pauli sum that maps real vectors to real vectors "
                         "(every c i^{|x&z|} real)");
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    t_dev = dev;
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) hipSetDevice(prev);
  }
};

// One ABI call on the handles it writes to or whose scratch it uses: each is
// taken for the duration of the call (a concurrent second call on any of
// them returns SV_EBUSY and changes nothing), then the device of the first
// is made current and checked for an earlier failure (SV_EDEVICE).
struct Call {
  sv_state* held[2] = {nullptr, nullptr};
  int n_held = 0;
  int rc = SV_OK;
  int prev_dev = -1;
  Call(sv_state* a, sv_state* b = nullptr) {
    for (sv_state* s : {a, b}) {
      if (!s) continue;
      int idle = 0;
      if (!s->busy.compare_exchange_strong(idle, 1)) {
        rc = fail(SV_EBUSY, "state handle is in use by another call (a handle is not re-entrant)");
        return;
      }
      held[n_held++] = s;
    }
    if (!n_held) return;
    const int dev = held[0]->device;
    t_dev = dev;
    if (hipGetDevice(&prev_dev) == hipSuccess && prev_dev != dev) hipSetDevice(dev);
    else prev_dev = -1;
    rc = device_check(dev);
  }
  ~Call() {
    if (prev_dev >= 0) hipSetDevice(prev_dev);
    for (int i = 0; i < n_held; ++i) held[i]->busy.store(0);
  }
};

static int get_cached_h(sv_state* s, const sv_pauli* p, const double* coef, int64_t n_terms, sv_hamiltonian** out) {
  int rc = validate_paulis(p, n_terms, s->n, "pauli sum");
  if (rc) return rc;
  rc = validate_finite(coef, n_terms, "coef");
  if (rc) return rc;
  uint64_t key = fnv(&n_terms, sizeof(n_terms));
  if (n_terms) {
    key = fnv(p, size_t(n_terms) * sizeof(sv_pauli), key);
    key = fnv(coef, size_t(n_terms) * sizeof(double), key);
  }
  // the hash only rejects quickly; a hit is confirmed on the terms themselves
  if (s->cached_h && s->cached_h->key == key && s->cached_h->n_terms == n_terms &&
      (n_terms == 0 || (std::memcmp(s->cached_h->src_p.data(), p, size_t(n_terms) * sizeof(sv_pauli)) == 0 &&
                        std::memcmp(s->cached_h->src_c.data(), coef, size_t(n_terms) * sizeof(double)) == 0))) {
    *out = s->cached_h;
    return SV_OK;
  }
  if (s->cached_h) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    hamiltonian_destroy(s->cached_h);
    s->cached_h = nullptr;
  }
  rc = hamiltonian_make(s->n, p, coef, n_terms, &s->cached_h);
  if (rc) return rc;
  s->cached_h->key = key;
  s->cached_h->src_p.assign(p, p + n_terms);
  s->cached_h->src_c.assign(coef, coef + n_terms);
  *out = s->cached_h;
  return SV_OK;
}

// ---------------------------------------------------------------------------
// rotations
// ---------------------------------------------------------------------------
struct RotPlan {
  std::vector<Run> runs;
  std::vector<RunData> data;
  std::vector<Pass> passes;
};

// grad_mode: 0 forward, 1 parameter gradient, 2 per-string gradient
static void plan_rotations(const sv_state* s, const sv_pauli* p, const double* phi, const double* dphi,
                           const int32_t* param, int64_t n_rot, bool reverse, int grad_mode, RotPlan& pl) {
  const PauliIn* pin = reinterpret_cast<const PauliIn*>(p);
  pl.runs = split_runs(pin, n_rot, param);
  pl.data.resize(pl.runs.size());
  for (size_t r = 0; r < pl.runs.size(); ++r)
    pl.data[r] = build_run_data(pl.runs[r], pin, phi, dphi, reverse ? grad_mode : 0);
  const int b = reverse ? tile_bits_two(s->dtype) : tile_bits_fwd(s->dtype);
  const int c = std::min(row_bits(s->dtype), s->n);
  const int slots_per_run = grad_mode == 1 ? 1 : 0;
  pl.passes = schedule(pl.runs, pl.data, pin, s->n, b, c, reverse, reverse && grad_mode ? kMaxPassSlots : 0,
                       slots_per_run, kMaxPassRuns, kMaxPassRecs);
}

// Launch a plan: forward (rev = false) or reverse with gradient partials.
// imag_count: see launch_tile_reverse (reverse sweeps only; NULL otherwise)
static int launch_rotations(sv_state* s, sv_state* lam, const RotPlan& pl, bool rev, int grad_mode,
                            double* partials, const double* imag_count = nullptr) {
  const int c = std::min(row_bits(s->dtype), s->n);
  // descriptors and records of every pass, one upload
  std::vector<RunDesc> descs;
  std::vector<RunRec> recs;
  std::vector<uint32_t> slot_maps;
  std::vector<SegDesc> segs;
  struct PassOff { size_t desc0; int nruns; size_t slot0; int nslots; size_t rec0; int nrecs; size_t seg0; int nsegs; };
  std::vector<PassOff> po;
  for (const Pass& ps : pl.passes) {
    PassOff o{descs.size(), int(ps.runs.size()), slot_maps.size(), 0, recs.size(), 0, segs.size(), 0};
    int local = 0;
    for (int ri : ps.runs) {
      const Run& r = pl.runs[ri];
      uint32_t slot;
      if (ps.tile) {
        slot = uint32_t(local);
        if (grad_mode == 1) {
          slot_maps.push_back(uint32_t(ri));
          local += 1;
        } else if (grad_mode == 2) {
          for (int k = 0; k < r.count; ++k) slot_maps.push_back(uint32_t(r.first + k));
          local += r.count;
        }
      } else {
        slot = grad_mode == 1 ? uint32_t(ri) : uint32_t(r.first);
      }
      descs.push_back(make_run_desc(r, pl.data[ri], ps.qmask, slot, grad_mode == 2, recs));
      if (ps.tile) descs.back().rec_off -= uint32_t(o.rec0);  // tile passes index their own records
    }
    o.nslots = local;
    o.nrecs = int(recs.size() - o.rec0);
    if (ps.tile) {
      // segments of the pass and each descriptor's walk for its segment
      std::vector<uint32_t> xl;
      for (size_t j = o.desc0; j < descs.size(); ++j) xl.push_back(uint32_t(descs[j].x_loc));
      const int fb = popc(ps.qmask);
      const std::vector<SegDesc> sp = segment_pass(xl, fb, kTileRegionBits);
      for (const SegDesc& sg : sp)
        for (uint32_t j = sg.first; j < sg.first + sg.count; ++j) {
          set_tile_walk(descs[o.desc0 + j], sg.wb_mask, fb);
          set_short_form(descs[o.desc0 + j], recs.data() + o.rec0);
        }
      segs.insert(segs.end(), sp.begin(), sp.end());
      o.nsegs = int(sp.size());
    }
    po.push_back(o);
  }
  if (recs.empty()) recs.push_back(RunRec{});
  Packer pk;
  const size_t o_desc = pk.add(descs.data(), descs.size() * sizeof(RunDesc));
  const size_t o_recs = pk.add(recs.data(), recs.size() * sizeof(RunRec));
  const size_t o_slot = pk.add(slot_maps.data(), slot_maps.size() * sizeof(uint32_t));
  const size_t o_segs = pk.add(segs.data(), segs.size() * sizeof(SegDesc));
  int rc = upload(s->staging, s->tables, pk, s->stream);
  if (rc) return rc;
  const RunDesc* d_desc = dptr<RunDesc>(s->tables, o_desc);
  const RunRec* d_recs = dptr<RunRec>(s->tables, o_recs);
  const uint32_t* d_slot = dptr<uint32_t>(s->tables, o_slot);
  const SegDesc* d_segs = dptr<SegDesc>(s->tables, o_segs);
  void* lam_amps = lam ? lam->amps : nullptr;
  for (size_t i = 0; i < pl.passes.size(); ++i) {
    const Pass& ps = pl.passes[i];
    if (ps.tile) {
      const FrameDesc fr = make_frame(ps.qmask, s->n, c);
      const uint64_t n_tb = uint64_t(1) << fr.n_comp;
      const int grid = int(std::min<uint64_t>(
          n_tb, uint64_t(std::min<int>(num_cus() * sweep_blocks_per_cu(s->dtype, rev), int(kPartialStride)))));
      hipError_t e;
      ProfScope prof(s->stream, rev ? kPTileRev : kPTileFwd, (rev ? 4.0 : 2.0) * s->bytes());
      if (!rev)
        e = launch_tile_forward(s->dtype, s->amps, fr, d_desc + po[i].desc0, d_recs + po[i].rec0,
                                d_segs + po[i].seg0, po[i].nsegs, n_tb, grid, s->stream);
      else
        e = launch_tile_reverse(s->dtype, grad_mode, s->amps, lam_amps, fr, d_desc + po[i].desc0,
                                d_recs + po[i].rec0, d_segs + po[i].seg0, po[i].nsegs, d_slot + po[i].slot0,
                                po[i].nslots, partials, kPartialStride, n_tb, grid, imag_count, s->stream);
      if (e != hipSuccess) return device_fail(std::string("tile pass launch: ") + hipGetErrorString(e));
    } else {
      const RunDesc& rd = descs[po[i].desc0];
      const Run& r = pl.runs[ps.runs[0]];
      uint64_t work;
      if (rd.mode == kRunEnum) work = uint64_t(1) << (s->n - rd.n_sup);
      else if (rd.mode == kRunFull) work = uint64_t(1) << (s->n - 1);
      else work = uint64_t(1) << s->n;
      (void)r;
      const double amp = s->bytes() / double(s->amp_count());
      const double touched = rd.mode == kRunDiag ? double(work) : 2.0 * double(work);
      ProfScope prof(s->stream, kPRunFull, touched * amp * 2.0 * (rev ? 2.0 : 1.0));
      const hipError_t e = launch_run_full(s->dtype, rev, rev ? grad_mode : 0, s->amps, lam_amps, rd, d_recs,
                                           partials, s->n, kPartialStride, full_grid(work), s->stream);
      if (e != hipSuccess) return device_fail(std::string("run launch: ") + hipGetErrorString(e));
    }
  }
  return SV_OK;
}

// ---------------------------------------------------------------------------
// Pauli-sum passes
// ---------------------------------------------------------------------------
static int dot_grid(const sv_state* s) { return full_grid(s->amp_count() / 4); }

// algorithmic bytes of one whole-state group pass: the amplitude pairs it
// reads (and, building lambda, the lambda pairs it reads and writes)
static double group_bytes(const sv_state* s, const GroupDesc& g, bool lambda) {
  const double amp = s->bytes() / double(s->amp_count());
  double touched;
  if (g.is_diag) touched = double(s->amp_count());
  else if (g.enumerated) touched = 2.0 * double(g.n_rec) * double(uint64_t(1) << (s->n - g.n_sup));
  else touched = double(s->amp_count());
  return touched * amp * (lambda ? 3.0 : 1.0);
}

// FP64 scratch of one expectation: the partial sums of its tile passes,
// whole-state group passes and norm/diagonal reductions, then four values
static size_t expect_scratch_doubles(const sv_state* s, const HTiling& ht, size_t* n_h) {
  const uint64_t n_tb = uint64_t(1) << ht.frames[0].n_comp;
  const uint32_t bpt = uint32_t(std::min<uint64_t>(n_tb, uint64_t(num_cus())));
  *n_h = ht.frames.size() * size_t(bpt) + ht.groups.size() * size_t(full_grid(s->amp_count() / 2));
  return *n_h + 3 * size_t(dot_grid(s)) + 4;
}

// The launches of an expectation (tables and diagonal already resident):
// part holds the partial sums (expect_scratch_doubles), sm four more
// doubles; every entry read is written first, so neither needs clearing.
// out_dev[0] = <psi|H|psi>/<psi|psi>, out_dev[1] = <psi|psi>
static int expect_launch(sv_state* s, const DevTiling* t, const double* diag, double* part, double* sm,
                         double* out_dev) {
  const HTiling& ht = t->host;
  const int T = int(ht.frames.size());
  const uint64_t n_tb = uint64_t(1) << ht.frames[0].n_comp;
  const uint32_t bpt = uint32_t(std::min<uint64_t>(n_tb, uint64_t(num_cus())));
  const size_t n_full = ht.groups.size();
  const int gfull = full_grid(s->amp_count() / 2);
  const int gdot = dot_grid(s);
  const size_t n_h = size_t(T) * bpt + n_full * size_t(gfull);
  hipError_t e;
  const uint4* blobs = dptr<uint4>(t->buf, t->o_blob);
  for (int tt = 0; tt < T; ++tt) {
    ProfScope prof(s->stream, kPTileHExp, s->bytes());
    e = launch_tile_expect(s->dtype, s->amps, ht.frames[tt], blobs + ht.blob_off[tt], n_tb, int(bpt),
                           part + size_t(tt) * bpt, s->stream);
    if (e != hipSuccess) return device_fail(std::string("expectation tiles: ") + hipGetErrorString(e));
  }
  size_t off = size_t(T) * bpt;
  for (size_t gi = 0; gi < n_full; ++gi) {
    ProfScope prof(s->stream, kPGroupFull, group_bytes(s, ht.groups[gi], false));
    e = launch_group_full(s->dtype, 0, s->amps, nullptr, ht.groups[gi], dptr<SubDesc>(t->buf, t->o_subs),
                          dptr<double2>(t->buf, t->o_coef), dptr<uint64_t>(t->buf, t->o_recs), s->n, gfull,
                          part + off, s->stream);
    if (e != hipSuccess) return device_fail(std::string("expectation group: ") + hipGetErrorString(e));
    off += size_t(gfull);
  }
  double* dpart = part + n_h;
  {
    ProfScope prof(s->stream, kPDot, s->bytes() * (diag ? 1.5 : 1.0));
    e = launch_dot(s->dtype, s->amps, nullptr, diag, s->amp_count(), gdot, dpart, s->stream);
  }
  if (e != hipSuccess) return device_fail("norm launch failed");
  ProfScope prof(s->stream, kPSmall, 0.0);
  HIP_TRY(launch_reduce_rows(part, 0, uint32_t(n_h), 1, sm, s->stream));
  HIP_TRY(launch_reduce_rows(dpart + 2 * gdot, 0, uint32_t(gdot), 1, sm + 1, s->stream));
  HIP_TRY(launch_reduce_rows(dpart + gdot, 0, uint32_t(gdot), 1, sm + 2, s->stream));
  HIP_TRY(launch_finish_energy(sm, 2, sm + 2, out_dev, s->stream));
  return SV_OK;
}

// out_dev[0] = <psi|H|psi>/<psi|psi>, out_dev[1] = <psi|psi>
static int expect_impl(sv_state* s, sv_hamiltonian* h, double* out_dev) {
  DevTiling* t = nullptr;
  int rc = tiling_get(h, s->dtype, 0, &t);
  if (rc) return rc;
  const double* diag = nullptr;
  rc = diag_get(h, s->stream, &diag);
  if (rc) return rc;
  size_t n_h = 0;
  const size_t need = expect_scratch_doubles(s, t->host, &n_h);
  rc = s->scratch.ensure((need + 8) * sizeof(double), s->stream);
  if (rc) return rc;
  double* part = static_cast<double*>(s->scratch.p);
  return expect_launch(s, t, diag, part, part + (need - 4), out_dev);
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free expectation (sv_expect_hamiltonian_noalloc):
// device memory held by the code object itself, one copy per device for the
// life of the process.  Host code never names the array (on the host its
// name is only a stand-in); it uses the device address looked up once per
// device, with that device current.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocDoubles = size_t(1) << 18;   // 2 MiB of FP64 partials
static __device__ __align__(256) double noalloc_scratch[kNoAllocDoubles];

static std::mutex g_noalloc_mu;
static double* g_noalloc_ptr[kMaxDevices] = {};

static int noalloc_scratch_of(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SV_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !p)
      return device_fail(std::string("hipGetSymbolAddress(noalloc scratch): ") + hipGetErrorString(e));
    g_noalloc_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return SV_OK;
}

// lam = H psi; energy_dev = (<psi|lam>/<psi|psi>, <psi|psi>)
static int lambda_impl(sv_state* s, sv_state* lam, sv_hamiltonian* h, double* energy_dev) {
  const int gdot = dot_grid(s);
  int rc = s->small.ensure(16 * sizeof(double), s->stream);
  if (rc) return rc;
  rc = s->scratch.ensure((3 * size_t(gdot) + 8) * sizeof(double), s->stream);
  if (rc) return rc;
  double* part = static_cast<double*>(s->scratch.p);
  double* sm = static_cast<double*>(s->small.p);
  // With real coefficients, count psi's nonzero imaginary parts; with none,
  // lambda is real and is built on the real-part tiling (one qubit more per
  // frame, fewer passes).  The choice of frames is the host's.  When the
  // caller has declared psi real (sv_set_real_hint) the real build is taken
  // without waiting, and its kernels check the device count themselves (a
  // nonzero count turns lambda into NaN); otherwise the host waits once for
  // the state's stream to read the count.  Only states whose real-part tiles
  // still give every compute unit a block (2^(n - kTileLamReal) >= CUs) take
  // the real build; smaller ones keep the complex build and skip the count.
  bool real = s->dtype == SV_R64;  // a real state: lambda is real (the sum was checked to be real)
  const double* guard = nullptr;
  if (!real && h->real && s->n > kTileLamReal && (uint64_t(1) << (s->n - kTileLamReal)) >= uint64_t(num_cus())) {
    {
      ProfScope prof(s->stream, kPDot, s->bytes());
      HIP_TRY(launch_imag_count(s->dtype, s->amps, s->amp_count(), gdot, part, s->stream));
    }
    ProfScope prof(s->stream, kPSmall, 0.0);
    HIP_TRY(launch_reduce_rows(part, 0, uint32_t(gdot), 1, sm + 15, s->stream));
    if (s->real_hint) {
      real = true;
      guard = sm + 15;
    } else {
      if (!s->host_word && hipHostMalloc(reinterpret_cast<void**>(&s->host_word), sizeof(double)) != hipSuccess) {
        s->host_word = nullptr;
        return fail(SV_ENOMEM, "pinned host word allocation failed");
      }
      *s->host_word = -1.0;
      HIP_TRY(hipMemcpyAsync(s->host_word, sm + 15, sizeof(double), hipMemcpyDeviceToHost, s->stream));
      HIP_TRY(hipStreamSynchronize(s->stream));
      real = *s->host_word == 0.0;
    }
  }
  DevTiling* t = nullptr;
  rc = tiling_get(h, s->dtype, real ? 2 : 1, &t);
  if (rc) return rc;
  const double* diag = nullptr;
  rc = diag_get(h, s->stream, &diag);
  if (rc) return rc;
  const HTiling& ht = t->host;
  const int T = int(ht.frames.size());
  // psi's largest amplitude exponent, per block: the fixed-point scale of the
  // tile passes (the third row of the scratch is free until the dot below)
  double* ep = part + 2 * size_t(gdot);
  if (T > 0) {
    ProfScope prof(s->stream, kPDot, s->bytes());
    HIP_TRY(launch_amp_exponent(s->dtype, s->amps, s->amp_count(), gdot, ep, s->stream));
  }
  for (int tt = 0; tt < T; ++tt) {
    const FrameDesc& fr = ht.frames[tt];
    const uint64_t n_tb = uint64_t(1) << fr.n_comp;
    const int grid = int(std::min<uint64_t>(n_tb, uint64_t(num_cus())));
    ProfScope prof(s->stream, kPTileHLam, (tt == 0 ? (diag ? 2.5 : 2.0) : 3.0) * s->bytes());
    const hipError_t e = launch_tile_lambda(s->dtype, tt == 0, real, s->amps, lam->amps, diag, fr,
                                            dptr<uint4>(t->buf, t->o_blob) + ht.blob_off[tt], n_tb, grid, guard, ep,
                                            gdot, s->stream);
    if (e != hipSuccess) return device_fail(std::string("lambda tile: ") + hipGetErrorString(e));
  }
  const int gfull = full_grid(s->amp_count() / 2);
  for (size_t gi = 0; gi < ht.groups.size(); ++gi) {
    ProfScope prof(s->stream, kPGroupFull, group_bytes(s, ht.groups[gi], true));
    const hipError_t e = launch_group_full(s->dtype, 2, s->amps, lam->amps, ht.groups[gi],
                                           dptr<SubDesc>(t->buf, t->o_subs), dptr<double2>(t->buf, t->o_coef),
                                           dptr<uint64_t>(t->buf, t->o_recs), s->n, gfull, nullptr, s->stream);
    if (e != hipSuccess) return device_fail(std::string("lambda group: ") + hipGetErrorString(e));
  }
  {
    ProfScope prof(s->stream, kPDot, 2.0 * s->bytes());
    HIP_TRY(launch_dot(s->dtype, s->amps, lam->amps, nullptr, s->amp_count(), gdot, part, s->stream));
  }
  ProfScope prof(s->stream, kPSmall, 0.0);
  HIP_TRY(launch_reduce_rows(part, 0, uint32_t(gdot), 1, sm, s->stream));
  HIP_TRY(launch_reduce_rows(part + gdot, 0, uint32_t(gdot), 1, sm + 1, s->stream));
  HIP_TRY(launch_finish_energy(sm, 1, sm + 1, energy_dev, s->stream));
  return SV_OK;
}

static int check_pair(sv_state* psi, sv_state* lam) {
  if (!psi || !lam) return fail(SV_EINVAL, "NULL state");
  if (psi == lam) return fail(SV_EINVAL, "psi and lam must be different states");
  if (psi->n != lam->n || psi->dtype != lam->dtype) return fail(SV_EINVAL, "psi and lam differ in n or dtype");
  if (psi->stream != lam->stream) return fail(SV_EINVAL, "psi and lam must share one stream");
  return SV_OK;
}

// common body of the adjoint calls; param == nullptr -> per-rotation gradient
// lam += sum_j alpha_j <P_j|psi> P_j (Eq. 12), then energy_dev = Rayleigh
// quotient of H_eff from <psi|lam>; ovl_dev (optional) gets the overlaps.
static int deflate_impl(sv_state* psi, sv_state* lam, const ProjArgs& pa, double* energy_dev, double* ovl_dev) {
  const int g = dot_grid(psi);
  int rc = psi->scratch.ensure((2 * size_t(pa.k) * size_t(g) + 3 * size_t(g) + 8) * sizeof(double), psi->stream);
  if (rc) return rc;
  rc = psi->small.ensure((16 + 2 * kMaxProj) * sizeof(double), psi->stream);
  if (rc) return rc;
  double* part = static_cast<double*>(psi->scratch.p);
  double* sm = static_cast<double*>(psi->small.p);
  double* ovl = sm + 16;
  {
    ProfScope prof(psi->stream, kPDot, (1.0 + pa.k) * psi->bytes());
    HIP_TRY(launch_overlaps(psi->dtype, psi->amps, pa, psi->amp_count(), g, part, psi->stream));
  }
  {
    ProfScope prof(psi->stream, kPSmall, 0.0);
    HIP_TRY(launch_reduce_rows(part, uint64_t(g), uint32_t(g), uint32_t(2 * pa.k), ovl, psi->stream));
  }
  {
    ProfScope prof(psi->stream, kPDot, (2.0 + pa.k) * psi->bytes());
    HIP_TRY(launch_deflate(psi->dtype, lam->amps, pa, ovl, psi->amp_count(), g, psi->stream));
  }
  {
    ProfScope prof(psi->stream, kPDot, 2.0 * psi->bytes());
    HIP_TRY(launch_dot(psi->dtype, psi->amps, lam->amps, nullptr, psi->amp_count(), g, part, psi->stream));
  }
  ProfScope prof(psi->stream, kPSmall, 0.0);
  HIP_TRY(launch_reduce_rows(part, 0, uint32_t(g), 1, sm, psi->stream));
  HIP_TRY(launch_reduce_rows(part + g, 0, uint32_t(g), 1, sm + 1, psi->stream));
  HIP_TRY(launch_finish_energy(sm, 1, sm + 1, energy_dev, psi->stream));
  if (ovl_dev)
    HIP_TRY(hipMemcpyAsync(ovl_dev, ovl, 2 * size_t(pa.k) * sizeof(double), hipMemcpyDeviceToDevice, psi->stream));
  return SV_OK;
}

// given (optional): the reverse plan of a resident rotation list, made by the
// caller with this call's angles (parameter mode)
static int adjoint_impl(sv_state* psi, sv_state* lam, sv_hamiltonian* h, const sv_pauli* rp, const double* phi,
                        int64_t n_rot, const int32_t* param, const double* dphi, int64_t n_params,
                        double* energy_dev, double* grad_dev, const ProjArgs* defl = nullptr,
                        double* ovl_dev = nullptr, RotPlan* given = nullptr) {
  int rc = validate_real_rotations(psi, rp, n_rot);
  if (rc) return rc;
  rc = validate_real_sum(psi, h);
  if (rc) return rc;
  rc = lambda_impl(psi, lam, h, energy_dev);
  if (rc) return rc;
  if (defl && defl->k > 0) {
    rc = deflate_impl(psi, lam, *defl, energy_dev, ovl_dev);
    if (rc) return rc;
  }
  const int grad_mode = param ? 1 : 2;
  RotPlan own;
  if (!given) plan_rotations(psi, rp, phi, dphi, param, n_rot, true, grad_mode, own);
  RotPlan& pl = given ? *given : own;
  // every run a real rotation (omega0 odd, no diagonal run): with psi and lam
  // real on entry they stay real, and the tile passes may take the real walk
  // once a device count of their nonzero imaginary parts reads zero
  bool real_runs = !pl.runs.empty() && psi->dtype != SV_R64;  // a real state is real by construction
  for (const RunData& d : pl.data) real_runs &= d.mode != kRunDiag && (d.omega0 & 1u);
  const double* imag_count = nullptr;
  if (real_runs) {
    const int g = dot_grid(psi);
    rc = psi->scratch.ensure((2 * size_t(g) + 8) * sizeof(double), psi->stream);
    if (rc) return rc;
    rc = psi->small.ensure(16 * sizeof(double), psi->stream);
    if (rc) return rc;
    double* part = static_cast<double*>(psi->scratch.p);
    double* sm = static_cast<double*>(psi->small.p);
    {
      ProfScope prof(psi->stream, kPDot, 2.0 * psi->bytes());
      HIP_TRY(launch_imag_count(psi->dtype, psi->amps, psi->amp_count(), g, part, psi->stream));
      HIP_TRY(launch_imag_count(lam->dtype, lam->amps, lam->amp_count(), g, part + g, psi->stream));
    }
    ProfScope prof(psi->stream, kPSmall, 0.0);
    HIP_TRY(launch_reduce_rows(part, 0, uint32_t(2 * g), 1, sm + 14, psi->stream));
    imag_count = sm + 14;
  }
  const size_t n_slots = grad_mode == 1 ? pl.runs.size() : size_t(n_rot);
  const size_t part_n = std::max<size_t>(n_slots, 1) * kPartialStride;
  rc = lam->scratch.ensure((part_n + n_slots + 8) * sizeof(double), lam->stream);
  if (rc) return rc;
  double* partials = static_cast<double*>(lam->scratch.p);
  double* slot_val = partials + part_n;
  {
    ProfScope prof(psi->stream, kPSmall, 0.0);
    HIP_TRY(launch_fill_f64(partials, part_n, 0.0, psi->stream));
  }
  rc = launch_rotations(psi, lam, pl, true, grad_mode, partials, imag_count);
  if (rc) return rc;
  ProfScope prof(psi->stream, kPSmall, 0.0);
  if (grad_mode == 2) {
    HIP_TRY(launch_reduce_rows(partials, kPartialStride, kPartialStride, uint32_t(n_rot), grad_dev, psi->stream));
    return SV_OK;
  }
  HIP_TRY(launch_reduce_rows(partials, kPartialStride, kPartialStride, uint32_t(n_slots), slot_val, psi->stream));
  // parameter i <- runs of parameter i, in list order
  std::vector<uint32_t> off(size_t(n_params) + 1, 0), idx, cnt(size_t(n_params), 0);
  for (const Run& r : pl.runs) cnt[size_t(r.param)]++;
  for (int64_t i = 0; i < n_params; ++i) off[size_t(i) + 1] = off[size_t(i)] + cnt[size_t(i)];
  idx.resize(off.back());
  std::vector<uint32_t> fill(off.begin(), off.end() - 1);
  for (size_t r = 0; r < pl.runs.size(); ++r) idx[fill[size_t(pl.runs[r].param)]++] = uint32_t(r);
  std::vector<double> w(idx.size(), 1.0);
  Packer pk;
  const size_t o_off = pk.add(off.data(), off.size() * sizeof(uint32_t));
  const size_t o_idx = pk.add(idx.data(), idx.size() * sizeof(uint32_t));
  const size_t o_w = pk.add(w.data(), w.size() * sizeof(double));
  // the tables buffer is still read by queued kernels; use lam's buffers
  rc = upload(lam->staging, lam->tables, pk, lam->stream);
  if (rc) return rc;
  HIP_TRY(launch_gather_slots(slot_val, dptr<uint32_t>(lam->tables, o_off), dptr<uint32_t>(lam->tables, o_idx),
                              dptr<double>(lam->tables, o_w), int(n_params), grad_dev, psi->stream));
  return SV_OK;
}

// ---------------------------------------------------------------------------
// resident rotation lists (sv_rotations)
// ---------------------------------------------------------------------------
struct sv_rotations {
  int n = 0;
  std::vector<PauliIn> p;             // the list, in application order
  std::vector<int32_t> param;         // parameter of each rotation
  std::vector<double> dphi;           // d phi_k / d theta_param
  int64_t n_params = 0;
  std::vector<Run> runs[2];           // split once: [0] forward, [1] per parameter (gradient)
  std::vector<Pass> passes[3][2];     // [dtype][reverse]: the last schedule made
  std::vector<uint32_t> key[3][2];    // what that schedule was made from (run_key)
  std::mutex mu;
};

// The schedule reads a run's tables only through their mode and record count
// (pass record budget, line fraction); equal keys give the same schedule.
static std::vector<uint32_t> run_key(const std::vector<RunData>& data) {
  std::vector<uint32_t> k(data.size());
  for (size_t i = 0; i < data.size(); ++i) k[i] = uint32_t(data[i].mode) << 24 | uint32_t(data[i].recs.size());
  return k;
}

// A call's plan from a resident list: the runs split once, this call's
// angles phi_k = dphi_k theta[param_k] in the run tables, and the schedule of
// the last call reused while the tables it depends on (run_key) are unchanged;
// otherwise it is made again from this call's tables.  The plan is the one the
// call would make for itself from (p, phi, param, dphi).
static void resident_plan(sv_rotations* r, const sv_state* s, const double* theta, bool reverse, RotPlan& pl) {
  const int dtype = s->dtype;
  std::vector<double> phi(r->p.size());
  for (size_t k = 0; k < phi.size(); ++k) phi[k] = r->dphi[k] * theta[r->param[k]];
  pl.runs = r->runs[reverse];
  pl.data.resize(pl.runs.size());
  for (size_t i = 0; i < pl.runs.size(); ++i)
    pl.data[i] = build_run_data(pl.runs[i], r->p.data(), phi.data(), reverse ? r->dphi.data() : nullptr,
                                reverse ? 1 : 0);
  std::vector<uint32_t> key = run_key(pl.data);
  std::lock_guard<std::mutex> lk(r->mu);
  if (r->key[dtype][reverse] != key || r->passes[dtype][reverse].empty()) {
    const int b = reverse ? tile_bits_two(dtype) : tile_bits_fwd(dtype);
    const int c = std::min(row_bits(dtype), s->n);
    r->passes[dtype][reverse] = schedule(pl.runs, pl.data, r->p.data(), s->n, b, c, reverse,
                                         reverse ? kMaxPassSlots : 0, reverse ? 1 : 0, kMaxPassRuns, kMaxPassRecs);
    r->key[dtype][reverse] = std::move(key);
  }
  pl.passes = r->passes[dtype][reverse];
}

static int check_resident(const sv_state* s, const sv_rotations* r, const double* theta) {
  if (!r) return fail(SV_EINVAL, "NULL rotation list");
  if (r->n != s->n) return fail(SV_EINVAL, "rotation list and state differ in n");
  int rc = validate_finite(theta, r->n_params, "theta");
  if (rc) return rc;
  return validate_real_rotations(s, reinterpret_cast<const sv_pauli*>(r->p.data()), int64_t(r->p.size()));
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* sv_last_error(void) { return g_err.c_str(); }

int sv_inject_device_failure(const char* msg) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  t_dev = dev;
  device_fail(std::string("injected: ") + (msg ? msg : ""));
  g_err.clear();
  return SV_OK;
}

int sv_profile_begin(void) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = true;
  return SV_OK;
}

int sv_profile_end(char* buf, size_t buflen) {
  std::vector<ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = false;
    recs.swap(g_prof.recs);
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  t_dev = dev;
  int rc = device_check(dev);
  if (rc) return rc;
  HIP_TRY(hipDeviceSynchronize());
  double ms[kPCount] = {}, bytes[kPCount] = {};
  long count[kPCount] = {};
  for (const ProfRec& r : recs) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) ms[r.cls] += t;
    bytes[r.cls] += r.bytes;
    count[r.cls] += 1;
  }
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (const ProfRec& r : recs) {
      g_prof.pool.push_back(r.a);
      g_prof.pool.push_back(r.b);
    }
  }
  std::string out = "{";
  bool first = true;
  for (int c = 0; c < kPCount; ++c) {
    if (!count[c]) continue;
    char tmp[256];
    snprintf(tmp, sizeof(tmp), "%s\"%s\": {\"launches\": %ld, \"ms\": %.6f, \"bytes\": %.1f}", first ? "" : ", ",
             kProfName[c], count[c], ms[c], bytes[c]);
    out += tmp;
    first = false;
  }
  out += "}";
  if (buf && buflen) {
    const size_t k = std::min(buflen - 1, out.size());
    std::memcpy(buf, out.data(), k);
    buf[k] = 0;
  }
  return SV_OK;
}

int sv_alloc(int n_qubits, int dtype, void* amps, size_t amps_bytes, void* hip_stream, sv_state** out) {
  if (!out) return fail(SV_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) return fail(SV_EINVAL, "n_qubits out of range");
  if (dtype != SV_C128 && dtype != SV_C64 && dtype != SV_R64) return fail(SV_EINVAL, "unknown dtype");
  if (!amps) return fail(SV_EINVAL, "amps is NULL");
  if (reinterpret_cast<uintptr_t>(amps) % 16) return fail(SV_EINVAL, "amps is not 16-byte aligned");
  const size_t need = (size_t(1) << n_qubits) * size_t(amp_bytes(dtype));
  if (amps_bytes < need) return fail(SV_EINVAL, "amps buffer smaller than 2^n amplitudes");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const int rc = device_check(dev);
  if (rc) return rc;
  sv_state* s = new sv_state();
  s->n = n_qubits;
  s->dtype = dtype;
  s->amps = amps;
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->device = dev;
  *out = s;
  g_err.clear();
  return SV_OK;
}

int sv_free(sv_state* s) {
  if (!s) return SV_OK;
  int rc;
  {
    Call call(s);
    if (call.rc == SV_EBUSY) return call.rc;
    rc = call.rc;
    // a failed device still gets its handle released; its stream is not waited for
    if (rc == SV_OK) hipStreamSynchronize(s->stream);
    if (s->cached_h) hamiltonian_destroy(s->cached_h);
    s->scratch.release();
    s->tables.release();
    s->small.release();
    s->staging.release();
    if (s->host_word) hipHostFree(s->host_word);
  }
  delete s;
  return rc;
}

int sv_set_stream(sv_state* s, void* hip_stream) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  Call call(s);
  if (call.rc) return call.rc;
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->stream = static_cast<hipStream_t>(hip_stream);
  return SV_OK;
}

int sv_set_real_hint(sv_state* s, int psi_is_real) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  Call call(s);
  if (call.rc) return call.rc;
  s->real_hint = psi_is_real != 0;
  return SV_OK;
}

int sv_prepare_hf(sv_state* s, uint64_t occ_mask) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  Call call(s);
  if (call.rc) return call.rc;
  if (occ_mask >> s->n) return fail(SV_EINVAL, "occ_mask has bits >= n");
  ProfScope prof(s->stream, kPFill, s->bytes());
  HIP_TRY(launch_fill_basis(s->dtype, s->amps, s->amp_count(), occ_mask, s->stream));
  return SV_OK;
}

int sv_apply_pauli_rotations(sv_state* s, const sv_pauli* p, const double* phi, int64_t n_rot) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  Call call(s);
  if (call.rc) return call.rc;
  int rc = validate_paulis(p, n_rot, s->n, "rotation");
  if (rc) return rc;
  rc = validate_finite(phi, n_rot, "phi");
  if (rc) return rc;
  rc = validate_real_rotations(s, p, n_rot);
  if (rc) return rc;
  if (n_rot == 0) return SV_OK;
  RotPlan pl;
  plan_rotations(s, p, phi, nullptr, nullptr, n_rot, false, 0, pl);
  return launch_rotations(s, nullptr, pl, false, 0, nullptr);
}

int sv_expect_pauli_sum(sv_state* s, const sv_pauli* p, const double* coef, int64_t n_terms, double* out_dev) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  Call call(s);
  if (call.rc) return call.rc;
  if (!out_dev) return fail(SV_EINVAL, "out_dev is NULL");
  sv_hamiltonian* h = nullptr;
  int rc = get_cached_h(s, p, coef, n_terms, &h);
  if (rc) return rc;
  return expect_impl(s, h, out_dev);
}

int sv_hamiltonian_create(int n_qubits, const sv_pauli* p, const double* coef, int64_t n_terms,
                          sv_hamiltonian** out) {
  if (!out) return fail(SV_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) return fail(SV_EINVAL, "n_qubits out of range");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const int rc = device_check(dev);
  if (rc) return rc;
  return hamiltonian_make(n_qubits, p, coef, n_terms, out);
}

int sv_hamiltonian_free(sv_hamiltonian* h) {
  if (!h) return SV_OK;
  DeviceGuard g(h->device);
  const int rc = device_check(h->device);
  if (rc == SV_OK) hipDeviceSynchronize();
  hamiltonian_destroy(h);
  return rc;
}

int sv_expect_hamiltonian(sv_state* s, const sv_hamiltonian* hc, double* out_dev) {
  if (!s || !hc) return fail(SV_EINVAL, "NULL argument");
  Call call(s);
  if (call.rc) return call.rc;
  if (!out_dev) return fail(SV_EINVAL, "out_dev is NULL");
  if (hc->n != s->n) return fail(SV_EINVAL, "Pauli sum and state differ in n");
  return expect_impl(s, const_cast<sv_hamiltonian*>(hc), out_dev);
}

int sv_expect_hamiltonian_noalloc(sv_state* s, const sv_hamiltonian* hc, double* out_dev) {
  if (!s || !hc) return fail(SV_EINVAL, "NULL argument");
  Call call(s);
  if (call.rc) return call.rc;
  if (!out_dev) return fail(SV_EINVAL, "out_dev is NULL");
  if (hc->n != s->n) return fail(SV_EINVAL, "Pauli sum and state differ in n");
  sv_hamiltonian* h = const_cast<sv_hamiltonian*>(hc);
  const DevTiling* t = nullptr;
  const double* diag = nullptr;
  {
    // the resident tables and diagonal must exist already: building them allocates
    std::lock_guard<std::mutex> lk(h->mu);
    if (!h->built[s->dtype][0] || (!h->diag_z.empty() && !h->diag_built))
      return fail(SV_EINVAL,
                  "the Pauli sum's expectation tables for this dtype are not built yet (one sv_expect_hamiltonian "
                  "call with a state of this dtype builds them)");
    t = &h->tilings[s->dtype][0];
    if (!h->diag_z.empty()) diag = static_cast<const double*>(h->diag_dev.p);
  }
  size_t n_h = 0;
  const size_t need = expect_scratch_doubles(s, t->host, &n_h);
  if (need > kNoAllocDoubles)
    return fail(SV_EINVAL, "the expectation needs " + std::to_string(need) + " FP64 partials, more than the " +
                               std::to_string(kNoAllocDoubles) + " of the allocation-free scratch");
  double* part = nullptr;
  int rc = noalloc_scratch_of(s->device, &part);
  if (rc) return rc;
  if (diag) HIP_TRY(hipStreamWaitEvent(s->stream, h->diag_ready, 0));
  return expect_launch(s, t, diag, part, part + (need - 4), out_dev);
}

int sv_adjoint_grad(sv_state* psi, sv_state* lam, const sv_pauli* hp, const double* hcoef, int64_t n_terms,
                    const sv_pauli* rp, const double* phi, int64_t n_rot, double* energy_dev, double* grad_dev) {
  int rc = check_pair(psi, lam);
  if (rc) return rc;
  Call call(psi, lam);
  if (call.rc) return call.rc;
  if (!energy_dev || (n_rot > 0 && !grad_dev)) return fail(SV_EINVAL, "NULL output");
  rc = validate_paulis(rp, n_rot, psi->n, "rotation");
  if (rc) return rc;
  rc = validate_finite(phi, n_rot, "phi");
  if (rc) return rc;
  sv_hamiltonian* h = nullptr;
  rc = get_cached_h(psi, hp, hcoef, n_terms, &h);
  if (rc) return rc;
  return adjoint_impl(psi, lam, h, rp, phi, n_rot, nullptr, nullptr, 0, energy_dev, grad_dev);
}

static int check_params(const int32_t* param, const double* dphi, int64_t n_rot, int64_t n_params) {
  if (n_params < 0) return fail(SV_EINVAL, "negative n_params");
  if (n_rot > 0 && (!param || !dphi)) return fail(SV_EINVAL, "NULL parameter map");
  for (int64_t k = 0; k < n_rot; ++k)
    if (param[k] < 0 || param[k] >= n_params)
      return fail(SV_EINVAL, "param_of_rot[" + std::to_string(k) + "] out of range");
  return validate_finite(dphi, n_rot, "dphi_dtheta");
}

int sv_adjoint_grad_params(sv_state* psi, sv_state* lam, const sv_pauli* hp, const double* hcoef, int64_t n_terms,
                           const sv_pauli* rp, const double* phi, int64_t n_rot, const int32_t* param,
                           const double* dphi, int64_t n_params, double* energy_dev, double* grad_theta_dev) {
  int rc = check_pair(psi, lam);
  if (rc) return rc;
  Call call(psi, lam);
  if (call.rc) return call.rc;
  if (!energy_dev || (n_params > 0 && !grad_theta_dev)) return fail(SV_EINVAL, "NULL output");
  rc = validate_paulis(rp, n_rot, psi->n, "rotation");
  if (rc) return rc;
  rc = validate_finite(phi, n_rot, "phi");
  if (rc) return rc;
  rc = check_params(param, dphi, n_rot, n_params);
  if (rc) return rc;
  sv_hamiltonian* h = nullptr;
  rc = get_cached_h(psi, hp, hcoef, n_terms, &h);
  if (rc) return rc;
  return adjoint_impl(psi, lam, h, rp, phi, n_rot, param, dphi, n_params, energy_dev, grad_theta_dev);
}

int sv_adjoint_grad_params_h(sv_state* psi, sv_state* lam, const sv_hamiltonian* hc, const sv_pauli* rp,
                             const double* phi, int64_t n_rot, const int32_t* param, const double* dphi,
                             int64_t n_params, double* energy_dev, double* grad_theta_dev) {
  int rc = check_pair(psi, lam);
  if (rc) return rc;
  Call call(psi, lam);
  if (call.rc) return call.rc;
  if (!hc) return fail(SV_EINVAL, "NULL Pauli sum");
  if (hc->n != psi->n) return fail(SV_EINVAL, "Pauli sum and state differ in n");
  if (!energy_dev || (n_params > 0 && !grad_theta_dev)) return fail(SV_EINVAL, "NULL output");
  rc = validate_paulis(rp, n_rot, psi->n, "rotation");
  if (rc) return rc;
  rc = validate_finite(phi, n_rot, "phi");
  if (rc) return rc;
  rc = check_params(param, dphi, n_rot, n_params);
  if (rc) return rc;
  return adjoint_impl(psi, lam, const_cast<sv_hamiltonian*>(hc), rp, phi, n_rot, param, dphi, n_params,
                      energy_dev, grad_theta_dev);
}

int sv_rotations_create(int n_qubits, const sv_pauli* p, int64_t n_rot, const int32_t* param_of_rot,
                        const double* dphi_dtheta, int64_t n_params, sv_rotations** out) {
  if (!out) return fail(SV_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_qubits < 1 || n_qubits > SV_MAX_QUBITS) return fail(SV_EINVAL, "n_qubits out of range");
  int rc = validate_paulis(p, n_rot, n_qubits, "rotation");
  if (rc) return rc;
  rc = check_params(param_of_rot, dphi_dtheta, n_rot, n_params);
  if (rc) return rc;
  sv_rotations* r = new (std::nothrow) sv_rotations();
  if (!r) return fail(SV_ENOMEM, "rotation list handle");
  r->n = n_qubits;
  r->n_params = n_params;
  const PauliIn* pin = reinterpret_cast<const PauliIn*>(p);
  r->p.assign(pin, pin + n_rot);
  r->param.assign(param_of_rot, param_of_rot + n_rot);
  r->dphi.assign(dphi_dtheta, dphi_dtheta + n_rot);
  r->runs[0] = split_runs(r->p.data(), n_rot, nullptr);
  r->runs[1] = split_runs(r->p.data(), n_rot, r->param.data());
  *out = r;
  return SV_OK;
}

int sv_rotations_free(sv_rotations* r) {
  delete r;
  return SV_OK;
}

int sv_apply_rotations_h(sv_state* s, sv_rotations* r, const double* theta) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  Call call(s);
  if (call.rc) return call.rc;
  int rc = check_resident(s, r, theta);
  if (rc) return rc;
  if (r->p.empty()) return SV_OK;
  RotPlan pl;
  resident_plan(r, s, theta, false, pl);
  return launch_rotations(s, nullptr, pl, false, 0, nullptr);
}

int sv_adjoint_grad_params_hr(sv_state* psi, sv_state* lam, const sv_hamiltonian* hc, sv_rotations* r,
                              const double* theta, double* energy_dev, double* grad_theta_dev) {
  int rc = check_pair(psi, lam);
  if (rc) return rc;
  Call call(psi, lam);
  if (call.rc) return call.rc;
  if (!hc) return fail(SV_EINVAL, "NULL Pauli sum");
  if (hc->n != psi->n) return fail(SV_EINVAL, "Pauli sum and state differ in n");
  rc = check_resident(psi, r, theta);
  if (rc) return rc;
  if (!energy_dev || (r->n_params > 0 && !grad_theta_dev)) return fail(SV_EINVAL, "NULL output");
  RotPlan pl;
  resident_plan(r, psi, theta, true, pl);
  return adjoint_impl(psi, lam, const_cast<sv_hamiltonian*>(hc), reinterpret_cast<const sv_pauli*>(r->p.data()),
                      nullptr, int64_t(r->p.size()), r->param.data(), r->dphi.data(), r->n_params, energy_dev,
                      grad_theta_dev, nullptr, nullptr, &pl);
}

int sv_adjoint_grad_params_deflated(sv_state* psi, sv_state* lam, const sv_hamiltonian* hc,
                                    const sv_state* const* proj, const double* alpha, int n_proj,
                                    const sv_pauli* rp, const double* phi, int64_t n_rot, const int32_t* param,
                                    const double* dphi, int64_t n_params, double* energy_dev, double* ovl_dev,
                                    double* grad_theta_dev) {
  int rc = check_pair(psi, lam);
  if (rc) return rc;
  Call call(psi, lam);
  if (call.rc) return call.rc;
  if (!hc) return fail(SV_EINVAL, "NULL Pauli sum");
  if (hc->n != psi->n) return fail(SV_EINVAL, "Pauli sum and state differ in n");
  if (!energy_dev || (n_params > 0 && !grad_theta_dev)) return fail(SV_EINVAL, "NULL output");
  if (n_proj < 0 || n_proj > kMaxProj) return fail(SV_EINVAL, "n_proj out of range (0..8)");
  if (n_proj > 0 && (!proj || !alpha)) return fail(SV_EINVAL, "NULL deflation states or weights");
  ProjArgs pa{};
  pa.k = n_proj;
  for (int j = 0; j < n_proj; ++j) {
    const sv_state* q = proj[j];
    if (!q) return fail(SV_EINVAL, "NULL deflation state");
    if (q == psi || q == lam) return fail(SV_EINVAL, "a deflation state is psi or lam");
    if (q->n != psi->n || q->dtype != psi->dtype) return fail(SV_EINVAL, "deflation state differs in n or dtype");
    if (q->device != psi->device) return fail(SV_EINVAL, "deflation state on another device");
    if (!std::isfinite(alpha[j])) return fail(SV_EINVAL, "alpha is not finite");
    pa.p[j] = q->amps;
    pa.alpha[j] = alpha[j];
  }
  rc = validate_paulis(rp, n_rot, psi->n, "rotation");
  if (rc) return rc;
  rc = validate_finite(phi, n_rot, "phi");
  if (rc) return rc;
  rc = check_params(param, dphi, n_rot, n_params);
  if (rc) return rc;
  return adjoint_impl(psi, lam, const_cast<sv_hamiltonian*>(hc), rp, phi, n_rot, param, dphi, n_params,
                      energy_dev, grad_theta_dev, &pa, ovl_dev);
}

int sv_overlap(const sv_state* a, const sv_state* b, double* out_dev) {
  if (!a || !b) return fail(SV_EINVAL, "NULL state");
  sv_state* s = const_cast<sv_state*>(b);
  Call call(s);
  if (call.rc) return call.rc;
  if (!out_dev) return fail(SV_EINVAL, "NULL output");
  if (a->n != b->n || a->dtype != b->dtype) return fail(SV_EINVAL, "states differ in n or dtype");
  if (a->device != b->device) return fail(SV_EINVAL, "states on different devices");
  ProjArgs pa{};
  pa.k = 1;
  pa.p[0] = a->amps;
  const int gd = dot_grid(s);
  int rc = s->scratch.ensure((2 * size_t(gd) + 8) * sizeof(double), s->stream);
  if (rc) return rc;
  double* part = static_cast<double*>(s->scratch.p);
  {
    ProfScope prof(s->stream, kPDot, 2.0 * s->bytes());
    HIP_TRY(launch_overlaps(s->dtype, s->amps, pa, s->amp_count(), gd, part, s->stream));
  }
  ProfScope prof(s->stream, kPSmall, 0.0);
  HIP_TRY(launch_reduce_rows(part, uint64_t(gd), uint32_t(gd), 2, out_dev, s->stream));
  g_err.clear();
  return SV_OK;
}

int sv_normalize(sv_state* s, double* norm2_dev) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  Call call(s);
  if (call.rc) return call.rc;
  const int gdot = dot_grid(s);
  int rc = s->scratch.ensure((3 * size_t(gdot) + 8) * sizeof(double), s->stream);
  if (rc) return rc;
  rc = s->small.ensure(16 * sizeof(double), s->stream);
  if (rc) return rc;
  double* part = static_cast<double*>(s->scratch.p);
  double* sm = static_cast<double*>(s->small.p);
  {
    ProfScope prof(s->stream, kPDot, s->bytes());
    HIP_TRY(launch_dot(s->dtype, s->amps, nullptr, nullptr, s->amp_count(), gdot, part, s->stream));
  }
  ProfScope prof(s->stream, kPSmall, 2.0 * s->bytes());
  HIP_TRY(launch_reduce_rows(part + gdot, 0, uint32_t(gdot), 1, sm + 2, s->stream));
  HIP_TRY(launch_scale(s->dtype, s->amps, s->amp_count(), sm + 2, s->stream));
  if (norm2_dev) HIP_TRY(hipMemcpyAsync(norm2_dev, sm + 2, sizeof(double), hipMemcpyDeviceToDevice, s->stream));
  return SV_OK;
}

int sv_gather_amplitudes(sv_state* s, const uint64_t* idx, int64_t count, double* out_dev) {
  if (!s) return fail(SV_EINVAL, "NULL state");
  Call call(s);
  if (call.rc) return call.rc;
  if (count < 0 || (count > 0 && (!idx || !out_dev))) return fail(SV_EINVAL, "bad arguments");
  for (int64_t i = 0; i < count; ++i)
    if (idx[i] >> s->n) return fail(SV_EINVAL, "index out of range");
  if (count == 0) return SV_OK;
  Packer pk;
  const size_t o = pk.add(idx, size_t(count) * sizeof(uint64_t));
  int rc = upload(s->staging, s->tables, pk, s->stream);
  if (rc) return rc;
  HIP_TRY(launch_gather_amps(s->dtype, s->amps, dptr<uint64_t>(s->tables, o), count, out_dev, s->stream));
  return SV_OK;
}

}  // extern "C"
