/*
 * q2sv -- state-vector simulation of UCCSD circuits on one MI355X (gfx950).
 *
 * C ABI of libq2sv.so.  Plain pointers and sizes only.  Every call returns an
 * int: SV_OK (0) on success, a negative SV_E* code on failure, with a
 * thread-local message in sv_last_error().  No call throws or exits.
 *
 * Conventions (Section 3.1 Eq. 1-2, Section 3.2 Eq. 6, Section 4.2 Eq. 7,
 * Section 5.1 Eq. 10-11, Algorithm 1):
 *   - A state on n qubits is 2^n complex amplitudes; qubit q is bit q of the
 *     amplitude index (little-endian).  Amplitudes are interleaved (re, im):
 *     complex128 (SV_C128, 16 bytes) or complex64 (SV_C64, 8 bytes).  A real
 *     state (SV_R64) stores only the real parts, FP64 (8 bytes): the
 *     amplitudes of a circuit of real rotations started from a basis state
 *     (every Trotterised UCC circuit: each of its strings has an odd number
 *     of Y factors, so each rotation is a real orthogonal matrix).  It takes
 *     only real rotations (odd popcount(x & z); others are SV_EINVAL), and
 *     its adjoint calls take only sums that map real vectors to real vectors
 *     (every c_t i^{popcount(x_t & z_t)} real; others are SV_EINVAL).
 *     Results equal those of the complex128 state (whose imaginary parts are
 *     then exactly zero) up to rounding order, with half the bytes moved.
 *   - A Pauli string is sv_pauli {x, z}: bit q of x is set when the factor on
 *     qubit q is X or Y, bit q of z when it is Z or Y.  The operator is
 *     P = i^{popcount(x & z)} X^x Z^z, the plain tensor product of the
 *     factors (Hermitian, P^2 = I).
 *   - A rotation is R(P, phi) = exp(-i phi P / 2).  The Trotter product of
 *     Eq. 11 is a list of rotations applied in list order; the paper's
 *     exp(i theta P) is R(P, -2 theta).
 *   - A Pauli sum (Eq. 1) is H = sum_t c_t P_t with real c_t.
 *
 * Memory and streams.  The caller owns the amplitude buffer (device memory,
 * for example a contiguous torch tensor) and the HIP stream.  Every call only
 * enqueues work on the state's stream and returns (except that the adjoint
 * calls, given a sum whose coefficients are all real and a state large
 * enough to fill the device with 13-qubit tiles (21 qubits and more on 256
 * compute units), wait once for that stream to learn whether psi is real,
 * which selects a real-arithmetic build of lambda, unless the caller has
 * declared psi real with sv_set_real_hint); outputs named *_dev are device
 * pointers to FP64 values written on that stream.  Host arrays passed to a
 * call are read before the call returns; the caller may free them
 * afterwards.  Distinct handles may be used concurrently on different
 * streams and host threads.
 *
 * Errors.
 *   SV_EINVAL   an argument is invalid; arguments are validated before any
 *               device work, and the state is untouched.
 *   SV_ENOMEM   a device or pinned allocation of the library's own scratch
 *               failed; nothing else is affected.
 *   SV_EDEVICE  a HIP launch or runtime call failed.  The failure is sticky
 *               per device: from then on every call that would use that
 *               device (sv_alloc and sv_hamiltonian_create included)
 *               returns SV_EDEVICE, with the first failure's message in
 *               sv_last_error(), and does no device work.  sv_free and
 *               sv_hamiltonian_free still release their handle (and return
 *               SV_EDEVICE).  A caller should drain its work and report.
 *   SV_EBUSY    a handle is not re-entrant: a call made while another call
 *               on the same state handle (a state it writes to or whose
 *               scratch it uses) is in progress on another host thread
 *               returns SV_EBUSY at once and changes nothing.
 */
#ifndef Q2SV_H
#define Q2SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sv_state sv_state;             /* opaque: one state vector      */
typedef struct sv_hamiltonian sv_hamiltonian; /* opaque: resident Pauli sum    */
typedef struct sv_rotations sv_rotations;     /* opaque: resident rotation list */
typedef struct { uint64_t x, z; } sv_pauli;

enum { SV_C128 = 0, SV_C64 = 1, SV_R64 = 2 };
enum { SV_OK = 0, SV_EINVAL = -1, SV_ENOMEM = -2, SV_EDEVICE = -3, SV_EBUSY = -4 };

/* Largest supported qubit count (a 2^34 complex128 state is 256 GiB). */
#define SV_MAX_QUBITS 34

/* Bind a caller-owned device buffer as an n-qubit state (Eq. 7).
 *   n_qubits   1..SV_MAX_QUBITS
 *   dtype      SV_C128, SV_C64 or SV_R64
 *   amps       device pointer, 16-byte aligned, at least 2^n amplitudes
 *   amps_bytes size of that buffer in bytes (checked against 2^n * 16 or 8)
 *   hip_stream hipStream_t on which all work of this handle is enqueued
 *              (NULL = the default stream)
 *   out        receives the handle
 * The library allocates only the handle and small scratch (reduction
 * partials, staged tables); it never frees amps.  The amplitudes are not
 * initialised: call sv_prepare_hf or write them yourself. */
int sv_alloc(int n_qubits, int dtype, void *amps, size_t amps_bytes, void *hip_stream,
             sv_state **out);

/* Release the handle and its scratch (waits for the handle's stream). */
int sv_free(sv_state *s);

/* Change the stream of a handle (later calls enqueue there). */
int sv_set_stream(sv_state *s, void *hip_stream);

/* Declare whether psi is real when an adjoint call starts (Algorithm 1's
 * lambda = H psi), for example after sv_prepare_hf and rotations whose
 * strings all have an odd number of Y factors (every UCC string).  With a
 * real declaration the adjoint calls build lambda with real arithmetic
 * without waiting for the stream; the kernels still count psi's nonzero
 * imaginary parts on the device, and if any is found the declaration was
 * wrong: lambda, the energy and the gradient come out NaN (never silently
 * wrong).  psi_is_real = 0 (the default) restores the checked choice with
 * its one stream wait.  The declaration stays until changed. */
int sv_set_real_hint(sv_state *s, int psi_is_real);

/* psi <- |occ_mask>, the Hartree-Fock determinant of Eq. 6 as a basis state
 * (occupation of qubit q = bit q).  occ_mask < 2^n. */
int sv_prepare_hf(sv_state *s, uint64_t occ_mask);

/* psi <- R(p[n_rot-1], phi[n_rot-1]) ... R(p[0], phi[0]) psi   (Eq. 11).
 * p, phi are host arrays of n_rot >= 0 entries; every (x | z) < 2^n and every
 * phi finite.  Consecutive strings with the same x that commute are applied
 * as one fused pass (their product is the rotation by the summed angle on
 * each amplitude pair); runs whose x-masks fit one LDS tile are applied in
 * one HBM pass.  The result equals the one-at-a-time product up to rounding. */
int sv_apply_pauli_rotations(sv_state *s, const sv_pauli *p, const double *phi, int64_t n_rot);

/* Expectation of a Pauli sum (Eq. 2).  Writes out_dev[0] = <psi|H|psi> /
 * <psi|psi> and out_dev[1] = <psi|psi>, both FP64, on the state's stream.
 * Strings are grouped by x: one read of psi serves every z-variant of an x.
 * The reduction order is fixed by n and the term list, so repeated calls are
 * bitwise identical. */
int sv_expect_pauli_sum(sv_state *s, const sv_pauli *p, const double *coef, int64_t n_terms,
                        double *out_dev);

/* Reverse-mode gradient (Algorithm 1) of E = <psi|H|psi> with respect to
 * every rotation angle.  lambda = H psi is summed in 64-bit fixed point
 * (each term rounded at a power-of-two scale set by psi's largest amplitude,
 * about 2^-50 of the largest term a pass can form), so the result does not depend on
 * the order in which concurrent wavefronts add: lambda, the energy and the
 * gradient are bitwise equal from run to run, and a request alone or among
 * concurrent ones.
 *   psi     on entry U|psi0> from sv_apply_pauli_rotations with the same list;
 *           on return approximately psi0 (the rotations are undone).
 *   lam     scratch state with the same n and dtype; on return U^dag H U psi0.
 *   hp, hc, n_terms  the Pauli sum H (host arrays)
 *   rp, phi, n_rot   the rotation list that produced psi (host arrays)
 *   energy_dev       device FP64[2]: <psi|H|psi>/<psi|psi>, <psi|psi>
 *   grad_dev         device FP64[n_rot]: dE/dphi_k = Im <lam_k|P_k|psi_k>,
 *                    with psi_k, lam_k taken right after rotation k. */
int sv_adjoint_grad(sv_state *psi, sv_state *lam, const sv_pauli *hp, const double *hc,
                    int64_t n_terms, const sv_pauli *rp, const double *phi, int64_t n_rot,
                    double *energy_dev, double *grad_dev);

/* As sv_adjoint_grad, but returns the gradient with respect to parameters
 * theta, where phi_k = dphi_dtheta[k] * theta[param_of_rot[k]]:
 *   grad_theta_dev[i] = sum_{k: param_of_rot[k] = i} dphi_dtheta[k] dE/dphi_k.
 * param_of_rot entries lie in [0, n_params).  Runs are split so that one run
 * has one parameter; on amplitude pairs where a run acts as the identity and
 * contributes nothing to the gradient, the pass skips work. */
int sv_adjoint_grad_params(sv_state *psi, sv_state *lam, const sv_pauli *hp, const double *hc,
                           int64_t n_terms, const sv_pauli *rp, const double *phi, int64_t n_rot,
                           const int32_t *param_of_rot, const double *dphi_dtheta,
                           int64_t n_params, double *energy_dev, double *grad_theta_dev);

/* Resident Pauli sums (Eq. 1): group and upload once, then evaluate many
 * times.  sv_expect_pauli_sum and sv_adjoint_grad* with host term arrays keep
 * the grouped form of the last sum per state and reuse it when a later call
 * passes the same terms (compared entry by entry); a resident handle makes
 * that sharing explicit and lets several states use one copy.
 *   sv_hamiltonian_create  p, coef: host arrays of n_terms >= 0 entries,
 *                          copied before return; every (x | z) < 2^n_qubits,
 *                          every coef finite; 1 <= n_qubits <= SV_MAX_QUBITS.
 *                          Groups the terms by x on the host; the device
 *                          tables and the FP64 diagonal vector (8 bytes per
 *                          amplitude) are built on first use, under a
 *                          per-handle lock, the diagonal on the first caller's
 *                          stream, which later callers on other streams wait
 *                          for.  One handle may serve states on several streams
 *                          and host threads of the device current at creation.
 *   sv_hamiltonian_free    waits for the device, then releases the handle.
 *   sv_expect_hamiltonian  as sv_expect_pauli_sum with the resident sum (same
 *                          n as the state).
 *   sv_adjoint_grad_params_h  as sv_adjoint_grad_params with the resident sum.
 * Errors as the calls they mirror; SV_EINVAL when the handle's n differs from
 * the state's. */
int sv_hamiltonian_create(int n_qubits, const sv_pauli *p, const double *coef, int64_t n_terms,
                          sv_hamiltonian **out);
int sv_hamiltonian_free(sv_hamiltonian *h);
int sv_expect_hamiltonian(sv_state *s, const sv_hamiltonian *h, double *out_dev);
int sv_adjoint_grad_params_h(sv_state *psi, sv_state *lam, const sv_hamiltonian *h,
                             const sv_pauli *rp, const double *phi, int64_t n_rot,
                             const int32_t *param_of_rot, const double *dphi_dtheta,
                             int64_t n_params, double *energy_dev, double *grad_theta_dev);

/* Resident rotation lists (Eq. 10-11: U(theta) = prod_k exp(-i phi_k P_k / 2)
 * with phi_k = dphi_dtheta[k] theta[param_of_rot[k]]; Algorithm 1 for the
 * gradient): split into runs once; the pass schedule of the last call per
 * amplitude type and direction is kept and reused while the run tables it was
 * made from keep their kinds and record counts (as for every nonzero theta_p
 * of a UCC list), so such a call only writes the angle tables of its theta.
 *   sv_rotations_create  p, param_of_rot, dphi_dtheta: host arrays of n_rot
 *                        >= 0 entries, copied before return; every (x | z) <
 *                        2^n_qubits, 0 <= param_of_rot[k] < n_params, every
 *                        dphi finite.  No device work.
 *   sv_rotations_free    releases the handle (host memory only).
 *   sv_apply_rotations_h as sv_apply_pauli_rotations with phi_k =
 *                        dphi_dtheta[k] theta[param_of_rot[k]]; theta: host,
 *                        n_params entries, finite.
 *   sv_adjoint_grad_params_hr  as sv_adjoint_grad_params_h with the resident
 *                        list and theta in place of (rp, phi, param_of_rot,
 *                        dphi_dtheta, n_params).
 * A call's plan equals the one the non-resident calls make from the same
 * (p, phi, param_of_rot, dphi_dtheta), so results agree with them bit for bit.
 * One handle may serve several states and threads (its kept schedules are
 * read and replaced under a lock).  Errors as the calls they mirror; SV_EINVAL when the list's
 * n differs from the state's, or a real state meets a string with an even
 * number of Y factors. */
int sv_rotations_create(int n_qubits, const sv_pauli *p, int64_t n_rot, const int32_t *param_of_rot,
                        const double *dphi_dtheta, int64_t n_params, sv_rotations **out);
int sv_rotations_free(sv_rotations *r);
int sv_apply_rotations_h(sv_state *s, sv_rotations *r, const double *theta);
int sv_adjoint_grad_params_hr(sv_state *psi, sv_state *lam, const sv_hamiltonian *h, sv_rotations *r,
                              const double *theta, double *energy_dev, double *grad_theta_dev);

/* For callers that cannot allocate device memory during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * sv_expect_hamiltonian with no allocation of any kind.  Its FP64 partial
 * sums live in a fixed array of the library's device code (2 MiB, one copy
 * per device for the life of the process) instead of the handle's scratch.
 *   Preconditions: the resident sum's expectation tables and diagonal for
 *   the state's dtype exist, i.e. sv_expect_hamiltonian has run once with
 *   this handle and a state of that dtype (building them allocates);
 *   otherwise SV_EINVAL.  A call whose partial sums would exceed the array
 *   (tile passes x blocks + whole-state group passes x blocks + reductions
 *   > 262144 values) returns SV_EINVAL before any device work.
 *   The array is shared by every call on a device and keeps the last call's
 *   contents (every value a call reads it writes first): two calls whose
 *   work overlaps on one device, on different streams or host threads, race
 *   and must be ordered by the caller.
 *   Output, reduction order and errors otherwise as sv_expect_hamiltonian;
 *   the two give bitwise identical results. */
int sv_expect_hamiltonian_noalloc(sv_state *s, const sv_hamiltonian *h, double *out_dev);

/* Variational quantum deflation (Section 5.1, Eq. 12): the k-th excited
 * state minimizes <psi|H_eff|psi> with
 *   H_eff = H + sum_{j < n_proj} alpha[j] |Psi_j><Psi_j|.
 * As sv_adjoint_grad_params_h with H replaced by H_eff: the adjoint sweep
 * (Algorithm 1) starts from lambda = H psi + sum_j alpha[j] <Psi_j|psi> Psi_j.
 *   proj     host array of n_proj states (0 <= n_proj <= 8): same n, dtype
 *            and device as psi, neither psi nor lam; read on psi's stream,
 *            so writes to them from another stream must be ordered first by
 *            the caller.  Their normalization is the caller's.
 *   alpha    host FP64[n_proj], finite (copied before return)
 *   energy_dev  device FP64[2]: <psi|H_eff|psi>/<psi|psi>, <psi|psi>
 *   ovl_dev     device FP64[2 n_proj] or NULL: <Psi_j|psi> (re, im) at the
 *               circuit output
 * n_proj = 0 gives the plain call.  Errors as sv_adjoint_grad_params_h, and
 * SV_EINVAL for a bad deflation list. */
int sv_adjoint_grad_params_deflated(sv_state *psi, sv_state *lam, const sv_hamiltonian *h,
                                    const sv_state *const *proj, const double *alpha, int n_proj,
                                    const sv_pauli *rp, const double *phi, int64_t n_rot,
                                    const int32_t *param_of_rot, const double *dphi_dtheta,
                                    int64_t n_params, double *energy_dev, double *ovl_dev,
                                    double *grad_theta_dev);

/* Overlap <a|b> = sum_k conj(a[k]) b[k], reduced in FP64 in a fixed order
 * (the overlap term of Eq. 12).  out_dev: device FP64[2] = (re, im).  a and
 * b share n, dtype and device; both are read on b's stream. */
int sv_overlap(const sv_state *a, const sv_state *b, double *out_dev);

/* psi <- psi / ||psi|| with the norm reduced in FP64 (the scale is applied in
 * the amplitude precision).  norm2_dev (device FP64[1], may be NULL)
 * receives ||psi||^2 before scaling. */
int sv_normalize(sv_state *s, double *norm2_dev);

/* psi[k] for a list of host indices, copied to a device FP64 array of
 * 2 * count values (re, im); used to check single amplitudes at scale. */
int sv_gather_amplitudes(sv_state *s, const uint64_t *idx, int64_t count, double *out_dev);

/* Kernel timing (Section 6.1 reports time per iteration; this gives it per
 * kernel class).  sv_profile_begin starts recording a HIP event pair around
 * every kernel the library launches, on the stream it is launched on, with
 * the algorithmic bytes the launch must move (state reads and writes, not
 * counting cache effects).  sv_profile_end waits for the device, writes a
 * JSON object {class: {"launches", "ms", "bytes"}} into buf (NUL-terminated,
 * truncated to buflen) and stops recording.  Process-wide; not re-entrant. */
int sv_profile_begin(void);
int sv_profile_end(char *buf, size_t buflen);

/* Message of the last failed call on this host thread ("" if none). */
const char *sv_last_error(void);

/* Mark the current device as failed, exactly as a failed HIP call would (see
 * SV_EDEVICE above), without touching the device.  For tests of a caller's
 * failure handling (draining, reporting); the mark lasts until the process
 * ends. */
int sv_inject_device_failure(const char *msg);

#ifdef __cplusplus
}
#endif

#endif /* Q2SV_H */
