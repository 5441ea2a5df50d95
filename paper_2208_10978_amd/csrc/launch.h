// Host-callable launchers of the gfx950 kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "q2sv_internal.h"

namespace q2sv {

// Tile widths (frame bits) per amplitude type and pass kind, chosen so the
// tiles fill at most 128 KiB of the 160 KiB LDS of a gfx950 compute unit.
constexpr int kTileFwdC128 = 13, kTileFwdC64 = 14;   // one state tile
constexpr int kTileTwoC128 = 12, kTileTwoC64 = 13;   // two tiles (psi and lam)
// The forward sweep of the 8-byte types runs on 64 KiB tiles (2^13
// amplitudes) so that two blocks share a compute unit: four wavefronts per
// SIMD hide the LDS and scalar-load latency of the per-run chains (real
// states at 28 qubits: 317 ms on one 128 KiB block, 163 ms; the 32-qubit
// complex64 stream: 151 -> 191 rotations/s).  complex128 keeps 2^13-amplitude
// tiles on one block (2^12 tiles and two blocks took 334 ms against 305 ms:
// more passes and whole-state runs).  The reverse sweep keeps one block of
// two 64 KiB tiles (two 32 KiB tiles and two blocks: 377 -> 456 ms).
constexpr int kTileSweepC128 = 13, kTileSweepC64 = 13, kTileSweepR64 = 13;
constexpr int kTileTwoR64 = 13;
constexpr int kSweepBlocks8 = 2;                     // blocks per compute unit, forward sweep, 8-byte types
constexpr int kTileLamC128 = 12, kTileLamC64 = 12;   // psi tile + FP64 lambda accumulator
constexpr int kTileLamReal = 13;                      // real parts of psi + one FP64 accumulator (real lambda)
constexpr int kTileThreads = 512;
constexpr int kTileRegionBits = 3;                   // 8 wavefronts own 8 regions of a segment
constexpr int kLambdaThreads = 1024;                 // 16 wavefronts share one tile
constexpr int kExpectThreads = 1024;                 // 16 wavefronts share one tile
constexpr int kMaxPassSlots = 96;                    // gradient slots per reverse tile pass (24 KiB of LDS cells)
constexpr int kMaxPassRuns = 1 << 16;                // runs per tile pass
constexpr int kMaxPassRecs = 1 << 20;                // run records per tile pass
constexpr uint32_t kPartialStride = 1024;            // max blocks of a gradient pass
static_assert(kPartialStride <= uint32_t(kLambdaThreads), "one amplitude-exponent partial per lambda thread");

hipError_t launch_fill_basis(int dtype, void* psi, uint64_t n_amp, uint64_t k, hipStream_t st);
hipError_t launch_run_full(int dtype, bool rev, int grad, void* psi, void* lam, const RunDesc& run,
                           const RunRec* recs, double* partials, int n, uint32_t nb_stride, int grid,
                           hipStream_t st);
// Tile passes: runs and recs are the pass's own descriptors and records
// (record offsets relative to recs); segs[0..n_segs) cover the runs in order
// and every descriptor's walk matches its segment's region bits.
hipError_t launch_tile_forward(int dtype, void* psi, const FrameDesc& fr, const RunDesc* runs, const RunRec* recs,
                               const SegDesc* segs, int n_segs, uint64_t n_tb, int grid, hipStream_t st);
// imag_count: device count of the nonzero imaginary parts of psi and lam
// (launch_imag_count), given only when every run of the list is a real
// rotation, or NULL; when it is zero, real runs take the real walk
hipError_t launch_tile_reverse(int dtype, int grad, void* psi, void* lam, const FrameDesc& fr,
                               const RunDesc* runs, const RunRec* recs, const SegDesc* segs, int n_segs,
                               const uint32_t* slot_map, int n_slots, double* partials, uint32_t nb_stride,
                               uint64_t n_tb, int grid, const double* imag_count, hipStream_t st);
// real: psi has no nonzero imaginary part and every coefficient of the sum is
// real; the frames are then those of a kTileLamReal-bit tiling and lambda is
// built from real parts only (always so for a real state, dtype 2).  guard
// (real builds of complex states only, may be NULL): device count of psi's
// nonzero imaginary parts; when it is not zero the pass writes NaN over
// lambda instead.  ep, n_ep: launch_amp_exponent's partials over psi (n_ep <=
// kLambdaThreads), which set the fixed-point scale.
hipError_t launch_tile_lambda(int dtype, bool first, bool real, const void* psi, void* lam, const double* diag,
                              const FrameDesc& fr, const uint4* blob, uint64_t n_tb, int grid, const double* guard,
                              const double* ep, int n_ep, hipStream_t st);
// partials[block] = number of the block's amplitudes with a nonzero imaginary part (grid blocks of 256)
hipError_t launch_imag_count(int dtype, const void* a, uint64_t n_amp, int grid, double* partials, hipStream_t st);
// partials[block] = largest exponent of |re| + |im| over the block's amplitudes (grid blocks of 256)
hipError_t launch_amp_exponent(int dtype, const void* a, uint64_t n_amp, int grid, double* partials, hipStream_t st);
hipError_t launch_tile_expect(int dtype, const void* psi, const FrameDesc& fr, const uint4* blob, uint64_t n_tb,
                              int grid, double* partials, hipStream_t st);
hipError_t launch_diag_build(double* d, uint64_t n_amp, const uint64_t* z, const double* c, int n_terms,
                             hipStream_t st);
hipError_t launch_group_full(int dtype, int mode, const void* psi, void* lam, const GroupDesc& g,
                             const SubDesc* subs, const double2* coef, const uint64_t* recbits, int n,
                             int grid, double* partials, hipStream_t st);
// partials[0..grid) = Re<a|b>, [grid..2grid) = <a|a>, [2grid..3grid) = sum d |a|^2
hipError_t launch_dot(int dtype, const void* a, const void* b, const double* d, uint64_t n_amp, int grid,
                      double* partials, hipStream_t st);
hipError_t launch_reduce_rows(const double* in, uint64_t stride, uint32_t len, uint32_t rows, double* out,
                              hipStream_t st);
hipError_t launch_finish_energy(const double* sums, int nh, const double* norm, double* out, hipStream_t st);
hipError_t launch_gather_slots(const double* slot_val, const uint32_t* off, const uint32_t* idx,
                               const double* weight, int n_out, double* out, hipStream_t st);
hipError_t launch_fill_f64(double* p, uint64_t n, double v, hipStream_t st);
hipError_t launch_scale(int dtype, void* psi, uint64_t n_amp, const double* norm2, hipStream_t st);
hipError_t launch_gather_amps(int dtype, const void* psi, const uint64_t* idx, int64_t count, double* out,
                              hipStream_t st);

// Deflation states (Eq. 12), passed by value: at most kMaxProj states.
constexpr int kMaxProj = 8;
struct ProjArgs {
  const void* p[kMaxProj];
  double alpha[kMaxProj];
  int k;
};
// partials[(2j) * grid + b], [(2j + 1) * grid + b] = Re, Im <P_j|psi> of block b
hipError_t launch_overlaps(int dtype, const void* psi, const ProjArgs& pa, uint64_t n_amp, int grid,
                           double* partials, hipStream_t st);
// lam += sum_j alpha_j ovl_j P_j (ovl: device FP64 (re, im) pairs)
hipError_t launch_deflate(int dtype, void* lam, const ProjArgs& pa, const double* ovl, uint64_t n_amp, int grid,
                          hipStream_t st);

// Bytes per amplitude: complex128 (0) 16, complex64 (1) and real FP64 (2) 8.
inline int amp_bytes(int dtype) { return dtype == 0 ? 16 : 8; }
// Low qubits that make a tile row one 128-byte line (always in a frame).
inline int row_bits(int dtype) { return dtype == 0 ? 3 : 4; }
// Tile widths follow the amplitude size (a real FP64 tile is laid out as a
// complex64 one).
inline int tile_bits_one(int dtype) { return dtype == 0 ? kTileFwdC128 : kTileFwdC64; }
// forward and reverse sweep tiles
inline int tile_bits_fwd(int dtype) { return dtype == 0 ? kTileSweepC128 : dtype == 1 ? kTileSweepC64 : kTileSweepR64; }
inline int tile_bits_two(int dtype) { return dtype == 0 ? kTileTwoC128 : dtype == 1 ? kTileTwoC64 : kTileTwoR64; }
inline int sweep_blocks_per_cu(int dtype, bool reverse) { return reverse || dtype == 0 ? 1 : kSweepBlocks8; }
inline int tile_bits_lambda(int dtype) { return dtype == 0 ? kTileLamC128 : kTileLamC64; }

}  // namespace q2sv
