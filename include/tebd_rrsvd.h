/*
 * tebd_rrsvd.h -- C interface of the MI355X TEBD bond-update library.
 *
 * Method: Tamascelli, Rosenbach, Plenio, "Improved scaling of Time-Evolving
 * Block-Decimation algorithm through Reduced-Rank Randomized Singular Value
 * Decomposition", arXiv:1504.00992.  The two-site TEBD update (Sec. II.B:
 * Theta of Eq. deftheta, the gate update of Eq. defupdatetheta, the blocked
 * matrix, extraction of the new Gamma and lambda) with the SVD replaced by
 * the reduced-rank randomized SVD (Sec. IV: Alg. 1 and steps i-iii).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Scalars: complex values are tebd_z, two interleaved IEEE doubles
 *   (re, im), the layout of C99 double _Complex and torch.complex128.
 * Memory: every pointer named "device" is HIP device memory on the current
 *   device, allocated and owned by the caller.  The library never allocates,
 *   frees or keeps device memory; scratch comes from the caller's workspace
 *   (size from tebd_workspace_size).  "host" pointers are read during the
 *   call only.
 * Streams: calls only enqueue work on `stream` (a hipStream_t, NULL = the
 *   null stream) and return; outputs are valid once the stream has been
 *   synchronised.  Calls on one stream run in order; concurrent calls need
 *   distinct workspaces.
 * Errors: arguments are checked on the host before anything is enqueued.  A
 *   non-zero tebd_status means nothing was enqueued; tebd_last_error() then
 *   names the offending argument (thread-local text).  Conditions found on
 *   the device never abort: they are OR-ed into per-problem status words
 *   (TEBD_DEV_* bits).
 * Layouts: matrices are row-major with a leading dimension (elements between
 *   rows).  Two-site gates are indexed row = i_k * d_{k+1} + i_{k+1}
 *   (Kronecker order); the blocked Theta has row i_k * chi_l + alpha and
 *   column i_{k+1} * chi_r + beta.
 * Sketch width: l = min(k + p, m, n).  The first QR step of Alg. 1 pivots
 *   columns and keeps the numerical range of the sketch (|R_jj| >
 *   1e-13 |R_00|), so at most that many singular values are returned.
 * Randomness: the Gaussian test matrix Omega (Sec. IV, Alg. 1, first step)
 *   is drawn by Philox4x32-10 (Salmon et al., SC'11).  Entry (r, c) of
 *   problem `pid` uses counter (r, c, pid, params.stream_id) and key
 *   (seed & 0xffffffff, seed >> 32); the first two output words x give
 *   u = (x + 1/2) 2^-32 and the complex normal
 *   z = sqrt(-2 ln u1) exp(2 pi i u2) / sqrt(2).
 */
#ifndef TEBD_RRSVD_H
#define TEBD_RRSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double re, im;
} tebd_z;

/* Host-detected errors; nothing is enqueued when one is returned. */
typedef enum {
  TEBD_OK = 0,
  TEBD_ERR_ARG = 1,       /* null pointer or value out of range          */
  TEBD_ERR_SHAPE = 2,     /* inconsistent dimensions / leading dims      */
  TEBD_ERR_WORKSPACE = 3, /* workspace missing, too small or misaligned  */
  TEBD_ERR_DEVICE = 4     /* a HIP call failed while enqueuing           */
} tebd_status;

/* Per-problem device status bits. */
enum {
  TEBD_DEV_NONFINITE = 1,     /* NaN/Inf met in the input or the factors     */
  TEBD_DEV_QR_FALLBACK = 2,   /* reserved: fast QR refused, fallback taken   */
  TEBD_DEV_JACOBI_NOCONV = 4, /* small SVD hit its sweep limit               */
  TEBD_DEV_LAMBDA_FLOOR = 8,  /* a lambda <= lambda_floor was not inverted   */
  TEBD_DEV_CHI_BOUND = 16,    /* chi_max (or l) binds before w <= trunc_eps  */
  TEBD_DEV_BAD_STATE = 32,    /* chi or d on the device out of range: the
                                 problem was skipped, the MPS left as it was */
  TEBD_DEV_RANK_RETRY = 64,   /* adaptive rank: stage 2 was needed (info)    */
  TEBD_DEV_ACC_CAPPED = 128   /* Accuracy Check: the basis reached its
                                 capacity min(chi_max + p, m, n) before the
                                 probes met the tolerance                    */
};

typedef struct {
  int32_t chi_max;      /* k: target rank and bond capacity, >= 1              */
  int32_t p;            /* oversampling, >= 0; sketch width l = min(k+p, m, n) */
  int32_t q;            /* power iterations of Alg. 1, >= 0                     */
  int32_t precision;    /* 0: FP64 throughout; 1: sketch and power-iteration
                           products in complex FP32 (QR, projection, small SVD
                           stay FP64)                                          */
  double trunc_eps;     /* keep the smallest chi' whose relative discarded
                           weight w = 1 - sum_{j<=chi'} s_j^2 / ||A||_F^2 is
                           <= trunc_eps (Sec. II.C, Eq. defdiscweigt); <= 0:
                           fixed rank min(chi_max, l)                          */
  double lambda_floor;  /* lambda <= floor is not inverted (its inverse is 0)  */
  uint64_t seed;        /* Philox key                                          */
  uint32_t stream_id;   /* Philox counter word 3 (e.g. a running sweep count)  */
  int32_t adaptive;     /* 0: fixed rank k = chi_max (Sec. IV, fixed-rank
                           problem).  1 (TEBD entry points only, trunc_eps > 0):
                           two-stage rank.  Stage 1 uses k1 = min(chi_max,
                           chi + max(4, ceil(chi/4))) with chi the bond
                           dimension before the update, and is kept when some
                           c <= k1 has w(c) <= trunc_eps; otherwise stage 2
                           repeats with k = chi_max, reusing the first Omega
                           columns.  This two-stage rule is this library's
                           own design: it stands in for the paper's Accuracy
                           Check (Sec. IV, Alg. 2, which grows the basis by
                           probe columns) with the exact Frobenius residual.
                           2: as 1 (same results), but the host reads back
                           how many bonds need stage 2 and skips that pass
                           when none does: the call then waits for the
                           stream once per sweep and cannot be captured in
                           a graph.
                           3 (TEBD entry points only, trunc_eps > 0): the
                           Accuracy Check of Sec. IV (Theorem 2, Alg. 2,
                           Fact 1).  The sketch starts with l = min(chi + p,
                           m, n) columns (chi: the bond dimension before the
                           update); after the first QR, blocks of
                           r = min(p, 16) Gaussian probes (the next columns
                           of the bond's test stream) estimate the range
                           error, max_i ||(I - QQ^H) A w_i||, against
                           sqrt(trunc_eps) ||A||_F / ((10/3) pi); while it is
                           larger the basis takes the probe products
                           A w_i (QR of [Q | A Omega_r]), up to
                           min(chi_max + p, m, n) columns (then
                           TEBD_DEV_ACC_CAPPED) and while l <= n - r; then
                           the power iterations and the truncation (chi' <=
                           chi_max).  The host waits for the stream once per
                           probe round                                        */
} tebd_params;

/* Fixed-capacity batch of MPS chains in Vidal form (Sec. II.A, Eq. defmps).
 * Site k of chain c holds d[k] matrices Gamma^[k]i of size chi_k x chi_{k+1},
 * stored padded at gamma[((c * n_sites + k) * d_max + i) * chi_max^2
 * + alpha * chi_max + beta].  Bond b (sites b, b+1) holds lambda^[b] at
 * lambda[(c * (n_sites - 1) + b) * chi_max + j], zero beyond chi_{b+1}.
 * chi[c * (n_sites + 1) + k] = chi_k with chi_0 = chi_N = 1.  Entries outside
 * the current chi must be zero on input; the library keeps them zero (an
 * update rewrites the updated bond's index only up to the larger of its old
 * and new dimension). */
typedef struct {
  int32_t n_chains, n_sites, d_max, chi_max;
  const int32_t* d; /* device [n_sites], 1 <= d[k] <= d_max                    */
  tebd_z* gamma;    /* device, see above                                       */
  double* lambda;   /* device, see above                                       */
  int32_t* chi;     /* device [n_chains][n_sites + 1]                          */
} tebd_mps;

/* Text of the last error on this thread ("" if none). */
const char* tebd_last_error(void);

/* Library version string. */
const char* tebd_version(void);

/* Bytes of workspace needed.
 *  - For tebd_bond_update / tebd_sweep / tebd_sweep_record: pass mps
 *    (non-NULL), batch = 0, m = n = NULL.  The size covers one sweep over
 *    every chain.  (tebd_sweep_adjoint: tebd_adjoint_workspace_size.)
 *  - For rrsvd_truncate: pass mps = NULL, the batch size and the host arrays
 *    m[batch], n[batch].
 * Returns TEBD_ERR_ARG / TEBD_ERR_SHAPE for invalid input. */
tebd_status tebd_workspace_size(const tebd_mps* mps, int64_t batch, const int64_t* m,
                                const int64_t* n, const tebd_params* prm, size_t* bytes);

/* Batched truncated SVD by RRSVD (Sec. IV: Alg. 1 with q power iterations
 * re-orthonormalised by Householder QR, then B = Q^H A, the SVD of B and
 * U = Q U_B; singular values sorted descending), followed by the truncation
 * rule on the relative discarded weight.  Drop-in for a truncated SVD call.
 *
 *  batch          number of problems (>= 1)
 *  m, n           host [batch]: rows / columns of problem b (>= 1)
 *  A              host [batch] of device pointers: m_b x n_b row-major,
 *                 leading dimension lda[b] >= n_b; read only
 *  lda            host [batch]
 *  omega          NULL: draw Omega from prm->seed (problem id b);
 *                 else host [batch] of device pointers to n_b x l_b row-major
 *                 test matrices (l_b = min(chi_max + p, m_b, n_b))
 *  U              host [batch] of device pointers: m_b x chi_max row-major,
 *                 leading dimension ldu >= chi_max; columns >= chi' zeroed
 *  S              host [batch] of device pointers: chi_max doubles, sorted
 *                 descending (not renormalised); entries >= chi' zeroed
 *  VH             host [batch] of device pointers: chi_max x n_b row-major,
 *                 leading dimension ldvh >= max n_b; rows >= chi' zeroed
 *  chi_kept       device [batch]: chi'
 *  disc_weight    device [batch]: relative discarded weight w of chi'
 *  dev_status     device [batch]: TEBD_DEV_* bits (overwritten)
 *  workspace      device, 256-byte aligned, ws_bytes from tebd_workspace_size
 */
tebd_status rrsvd_truncate(int64_t batch, const int64_t* m, const int64_t* n,
                           const tebd_z* const* A, const int64_t* lda,
                           const tebd_z* const* omega, const tebd_params* prm,
                           tebd_z* const* U, int64_t ldu, double* const* S,
                           tebd_z* const* VH, int64_t ldvh, int32_t* chi_kept,
                           double* disc_weight, int32_t* dev_status, void* workspace,
                           size_t ws_bytes, void* stream);

/* rrsvd_truncate for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and random stream as rrsvd_truncate, without the
 * workspace: scratch is a static device array of the library, 64 MiB per
 * device, held by every device the library runs on until the process ends.
 * The call allocates nothing (no hipMalloc, hipFree or pinned host buffer):
 * problem descriptors are written by a kernel from its arguments, and the
 * factorisation size classes run in order on `stream`.
 *  - A batch whose rrsvd_truncate workspace (tebd_workspace_size with
 *    mps = NULL) exceeds 64 MiB is refused with TEBD_ERR_WORKSPACE before
 *    anything is enqueued.
 *  - Every call on one device shares that device's scratch, which keeps the
 *    last call's contents (no part of it needs to start at zero).  Calls
 *    that overlap on one device race: serialise them (one stream, or events).
 *  - Outputs are valid once `stream` has been synchronised. */
tebd_status rrsvd_truncate_noalloc(int64_t batch, const int64_t* m, const int64_t* n,
                                   const tebd_z* const* A, const int64_t* lda,
                                   const tebd_z* const* omega, const tebd_params* prm,
                                   tebd_z* const* U, int64_t ldu, double* const* S,
                                   tebd_z* const* VH, int64_t ldvh, int32_t* chi_kept,
                                   double* disc_weight, int32_t* dev_status, void* stream);

/* One two-site update of bond `bond` (sites bond, bond+1) of chain `chain`
 * (Sec. II.B): Theta from Gamma-lambda-Gamma (Eq. deftheta), the gate
 * (Eq. defupdatetheta), the blocked matrix, its RRSVD truncation to chi',
 * lambda' = s / ||s|| (renormalised, Sec. II.C) and the new Gamma by
 * lambda^-1 reabsorption: Gamma'^[k]i_{a g} = U_{(i a), g} / lambda^[k-1]_a,
 * Gamma'^[k+1]j_{g b} = V^H_{g, (j b)} / lambda^[k+1]_b (lambda outside the
 * chain = 1; lambda <= lambda_floor gives 0 and sets TEBD_DEV_LAMBDA_FLOOR).
 *
 *  mps          the chain batch (updated in place on the device)
 *  gate         device: (d_k d_{k+1}) x (d_k d_{k+1}) complex, row-major
 *               with leading dimension d_max^2
 *  disc_weight  device [1]: relative discarded weight
 *  dev_status   device [1]: TEBD_DEV_* bits (overwritten)
 *  Omega problem id: chain * (n_sites - 1) + bond. */
tebd_status tebd_bond_update(const tebd_mps* mps, int32_t chain, int32_t bond,
                             const tebd_z* gate, const tebd_params* prm, double* disc_weight,
                             int32_t* dev_status, void* workspace, size_t ws_bytes,
                             void* stream);

/* One sweep of non-overlapping two-site gates (Sec. II.C, Eq. defst3rd: the
 * bonds of one parity commute and are updated together), over every chain.
 *
 *  parity             0: bonds 0, 2, 4, ...;  1: bonds 1, 3, 5, ...
 *  gates              device: gate of bond b of chain c at
 *                     gates + c * gate_chain_stride + b * d_max^4, each laid
 *                     out as in tebd_bond_update
 *  gate_chain_stride  elements between chains' gate sets (0: shared)
 *  disc_weight        device [n_chains][n_sites - 1]: written for the bonds
 *                     of this parity
 *  dev_status         device [n_chains][n_sites - 1]: same
 *  Omega problem id of bond b of chain c: c * (n_sites - 1) + b. */
tebd_status tebd_sweep(const tebd_mps* mps, const tebd_z* gates, int64_t gate_chain_stride,
                       int32_t parity, const tebd_params* prm, double* disc_weight,
                       int32_t* dev_status, void* workspace, size_t ws_bytes, void* stream);

/* Reverse mode.  The paper does not differentiate the bond update; these
 * entry points give the derivative of the map it defines, for gradients of
 * observables with respect to the gates (and, through exp(-i tau h_b), the
 * Hamiltonian couplings).  Cotangent convention: for a real loss L and a
 * complex entry z = x + i y the cotangent is dL/dx + i dL/dy; for a real
 * entry it is dL/dx.  Cotangent arrays use the layouts of tebd_mps and of
 * the gates.
 *
 * A time step is replayed sweep by sweep with tebd_sweep_record, which keeps
 * a copy of the state before each sweep (made by the caller) and the tape,
 * then undone in reverse order with tebd_sweep_adjoint. */

/* Bytes of workspace for tebd_sweep_adjoint on `mps` under `prm`; a
 * workspace of this size also serves tebd_sweep and tebd_sweep_record. */
tebd_status tebd_adjoint_workspace_size(const tebd_mps* mps, const tebd_params* prm,
                                        size_t* bytes);

/* Bytes of the tape of one recorded sweep of `mps` under `prm` (either
 * parity). */
tebd_status tebd_tape_size(const tebd_mps* mps, const tebd_params* prm, size_t* bytes);

/* tebd_sweep (same arguments, same results, same random stream) that also
 * writes, for every bond, what its adjoint needs into `tape` (device,
 * 256-byte aligned, tape_bytes >= tebd_tape_size): the bond's geometry and
 * every singular triplet its RRSVD computed, kept or not, as plain U, s and
 * V^H before renormalisation and reabsorption. */
tebd_status tebd_sweep_record(const tebd_mps* mps, const tebd_z* gates, int64_t gate_chain_stride,
                              int32_t parity, const tebd_params* prm, double* disc_weight,
                              int32_t* dev_status, void* tape, size_t tape_bytes,
                              void* workspace, size_t ws_bytes, void* stream);

/* Adjoint of one recorded sweep (every bond of the parity, every chain).
 *
 *  mps_in        the state before the recorded sweep (read only; the
 *                caller's copy), with the same capacities as when recorded
 *  gates, gate_chain_stride, parity, prm
 *                as passed to tebd_sweep_record (prm->lambda_floor, chi_max
 *                and p are used)
 *  tape          device: written by tebd_sweep_record for this sweep
 *  gamma_bar     device, layout of mps.gamma: on entry the cotangent of the
 *                state after the sweep, on return that of the state before
 *                it (sites the sweep did not touch are left as they are;
 *                entries outside the bond dimensions are written as zero)
 *  lambda_bar    device, layout of mps.lambda: same
 *  gate_bar      device, layout of the gates: the cotangent of each bond's
 *                gate is added to it (with a zero chain stride every chain
 *                adds to the shared gate)
 *  dev_status    device [n_chains][n_sites - 1]: for the bonds of this
 *                parity 0, or TEBD_DEV_BAD_STATE when the tape does not
 *                describe that bond of mps_in (the bond is then skipped)
 *
 * Per bond (Sec. II.B undone): the cotangents of Gamma'_k, Gamma'_k+1 are
 * divided by lambda_l, lambda_r (the reabsorption), that of lambda' goes
 * through the renormalisation; the SVD adjoint couples the kept triplets
 * to every triplet the RRSVD computed (those enter with zero cotangent),
 * with 1/(s_j^2 - s_i^2) broadened to D/(D^2 + eta^2), eta = 1e-12 s_1^2,
 * and the rest of the spectrum through the projector terms
 * (I - U U^H) Ubar S^-1 V^H + U S^-1 Vbar^H (I - V V^H); then
 * Theta-bar = G^H Abar, Gbar += Abar Theta^H, and back through Eq. deftheta.
 * Bonds are independent within a sweep; all sums have a fixed order. */
tebd_status tebd_sweep_adjoint(const tebd_mps* mps_in, const tebd_z* gates,
                               int64_t gate_chain_stride, int32_t parity, const tebd_params* prm,
                               const void* tape, size_t tape_bytes, tebd_z* gamma_bar,
                               double* lambda_bar, tebd_z* gate_bar, int32_t* dev_status,
                               void* workspace, size_t ws_bytes, void* stream);

/* Per-kernel timing with HIP events, for the per-phase split of the update
 * (the paper's profile of the two-site update, Sec. V.B).  Off by default.
 * While on, each phase of the bond update (Theta and gate, Omega, each
 * sketch product, each QR, the small SVD, ...) and, inside it, each kernel
 * launch of the library is bracketed by two events recorded on the launch
 * stream.  tebd_profile_enable(0 or 1) also discards what was recorded so
 * far; call it and the profiled entry points from one host thread.
 * tebd_profile_read waits for the recorded events and writes, for up to
 * `capacity` kinds, the kind's name (static string), the summed elapsed
 * milliseconds and the number of launches; *count receives the number of
 * kinds written.  Phase kinds come first ("qr", "sketch_AH_Q", ...), then
 * kernel kinds, named by the kernel instantiation as profiler tools print
 * it without the namespace ("k_qr_reg<512, 8, false>", "k_gate", ...).  The
 * records are then discarded. */
tebd_status tebd_profile_enable(int32_t on);
tebd_status tebd_profile_read(int32_t capacity, const char** names, double* ms, int64_t* launches,
                              int32_t* count);

/* Autotune cache, the only state the library keeps between calls (read by
 * every launch, written only by these setters, which must not run while
 * another thread enqueues work).  It picks the tile shape of the sketch,
 * power-iteration and projection products of Alg. 1 and Sec. IV step i per
 * launch, from the largest problem of the batch: its row count (bucketed
 * as <= 128, 256, 512, 1024, 2048, 8192) and sketch width (<= 32, 64, 80,
 * 128, 256).  variant 0: 32 x 32 output tiles (the default, also for unset
 * entries); 1: 64 x 64 tiles; 2: 16 x 16 tiles, each split over the
 * contraction depth between the four wavefronts of its workgroup; -1
 * unsets.  precision 1 (complex FP32 products) has variant 0 only.
 * precision 2 is the table of the TEBD entry points' FP64 products: it is
 * read under the MPS capacities (d_max * chi_max rows, chi_max + p width)
 * instead of a batch's bounds, so that every rank mode, graph capture
 * included, takes the same variant (precision 0 serves rrsvd_truncate).
 * Variants 0 and 1 give identical results (the same K order per output
 * element); variant 2 adds four partial sums over interleaved k-steps, so
 * its results differ from theirs by rounding only.  The package's
 * autotune module times the variants on synthetic batches and keeps its
 * choices in a JSON file.
 * tebd_tune_set: TEBD_ERR_ARG for an unknown precision or variant,
 * TEBD_ERR_SHAPE for sizes outside the buckets.
 * tebd_tune_get: the entry (-1: unset), or -1 for invalid arguments. */
tebd_status tebd_tune_set(int32_t precision, int32_t max_rows, int32_t width, int32_t variant);
int32_t tebd_tune_get(int32_t precision, int32_t max_rows, int32_t width);

/* Size class, hence kernel, that a factorisation of the given shape runs
 * in (a planning query; no device work).  factorization 0: the Householder
 * QR of a rows x l sketch (the class follows the sketch width l the problem
 * started with); 1: the small SVD of an l x l factor (rows is ignored).
 * QR classes: 0 k_qr_reg<512, 8, *>, 1 k_qr_reg<1024, 12, *>, 2 k_qr_lds,
 * 3 k_qr_glb; small-SVD classes: 0 k_svd_pairs<256, 0>, 1 k_svd_pairs<512, 1>,
 * 2 k_small_svd<1024, 2, true>, 3 k_small_svd<1024, 4, false>.  Returns -1
 * for sizes outside [1, 8192] x [1, 256] or an unknown factorization. */
int32_t tebd_size_class(int32_t factorization, int32_t rows, int32_t l);

#ifdef __cplusplus
}
#endif

#endif /* TEBD_RRSVD_H */
