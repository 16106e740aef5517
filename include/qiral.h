/*
 * qiral.h -- C ABI of the MI355X (gfx950) even-odd Wilson-Dirac library.
 *
 * The problem statement follows the goal of the paper (Barthou et al.,
 * arXiv:1401.2039, Sec. 2): xx[L (x) C (x) S] = Dirac^{-1} * bb[L (x) C (x) S],
 * with Dirac the Wilson operator of Fig. "dirac", solved by the CGNR template
 * (Fig. "CG") composed with the Schur-complement template ("schur").  The
 * paper's generated function takes bb and xx and keeps every other constant
 * (lattice, kappa, links) global; here those constants live in an opaque
 * lattice handle.
 *
 * Conventions (all calls):
 *   dims[4] = {Lx, Ly, Lz, Lt}; every L_mu must be even and >= 2 (the
 *   checkerboard index needs even extents).  Direction mu = 0..3 = x, y, z, t.
 *   Periodic boundaries in all four directions (Fig. "id": isPeriodic(L)).
 *   Parity of a site = (x + y + z + t) mod 2, even = 0.
 *
 *   Canonical gauge field: device memory, complex128 (re, im interleaved
 *   doubles), index order [t][z][y][x][mu][row][col]; U[x][mu] is the link
 *   from x to x + mu_hat; the backward link is its adjoint one site back.
 *   Canonical spinor field: device memory, complex128, index order
 *   [rhs][t][z][y][x][colour][spin] (spin fastest).
 *
 *   Internal ("packed") fields are opaque device buffers whose size is given
 *   by qiral_field_bytes().  A half-field holds the sites of one parity; a
 *   full field is the even half followed by the odd half; nrhs fields follow
 *   one another.  Storage classes: QIRAL_F64 (complex128), QIRAL_F32
 *   (complex64) and QIRAL_F16S (FP16 with one FP32 scale per site).
 *
 *   Streams: every call that takes a stream enqueues its GPU work on it and
 *   returns without waiting, except qiral_lattice_create, qiral_solve and
 *   qiral_solve_batch, which synchronise the stream before returning.  A NULL
 *   stream is the default stream.
 *
 *   Errors: every call returns a status.  All argument checks run before any
 *   HIP call, so an invalid call has no effect on the device.  No C++
 *   exception crosses the ABI.  qiral_last_error() gives a thread-local
 *   description of the last failure.
 *
 *   Memory: the caller owns every device buffer -- canonical and packed fields,
 *   the packed link stores, the solver workspace and the network's memory --
 *   sized by qiral_field_bytes, qiral_gauge_bytes, qiral_solve_workspace_bytes
 *   and qiral_nn_bytes.  The library allocates no device memory.  A lattice
 *   handle holds host-side state only: the geometry, kappa, mu, pointers to the
 *   caller's link stores, and what qiral_lattice_create makes once so that
 *   later calls allocate nothing: a 224 KiB pinned host buffer for the solver's
 *   convergence polls and four HIP events.  Calls on one handle must not
 *   overlap in time (they share the poll buffer and events).
 */
#ifndef QIRAL_H
#define QIRAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

struct ihipStream_t;
typedef struct ihipStream_t *qiral_stream_t; /* same type as hipStream_t */

/* The enums below are 32-bit integers.  C++ gets them with that underlying
 * type, so every int32_t value a caller passes is a value of the enum type and
 * reaches the entry point's own check (which rejects those out of range). */
#ifdef __cplusplus
#define QIRAL_ENUM enum : int32_t
#else
#define QIRAL_ENUM enum
#endif

typedef QIRAL_ENUM {
  QIRAL_OK = 0,
  QIRAL_ERR_INVALID_ARG = 1,   /* null pointer, bad enum, nrhs < 1, ...            */
  QIRAL_ERR_BAD_DIMS = 2,      /* an extent odd or < 2, or the lattice too large    */
  QIRAL_ERR_UNSUPPORTED = 3,   /* valid request the library does not implement      */
  QIRAL_ERR_HIP = 4,           /* a HIP runtime call failed (text in last_error)    */
  QIRAL_ERR_NOT_CONVERGED = 5, /* tolerance not met within maxiter; x and info hold
                                  the last iterate and its residual                */
  QIRAL_ERR_NONFINITE = 6,     /* a NaN or Inf appeared in a reduction              */
  QIRAL_ERR_WORKSPACE = 7      /* workspace missing or smaller than its size query  */
} qiral_status;

typedef QIRAL_ENUM { QIRAL_F64 = 0, QIRAL_F32 = 1, QIRAL_F16S = 2 } qiral_prec;
typedef QIRAL_ENUM { QIRAL_RECON18 = 18, QIRAL_RECON12 = 12 } qiral_recon;
typedef QIRAL_ENUM { QIRAL_EVEN = 0, QIRAL_ODD = 1, QIRAL_FULL = 2 } qiral_subset;
typedef QIRAL_ENUM {
  QIRAL_OP_D = 0,        /* full-lattice D = A - kappa H (A = 1 + 2 i kappa mu g5)  */
  QIRAL_OP_DDAG = 1,     /* D^dagger = A^dagger - kappa H^dagger                    */
  QIRAL_OP_SCHUR = 2,    /* odd-site Schur complement S = A - kappa^2 H_oe A^-1 H_eo */
  QIRAL_OP_SCHUR_DAG = 3 /* S^dagger (see qiral_apply_M)                             */
} qiral_op;
/* The system a solver runs on (template chain "solver schur" or the solver on D
 * itself, Sec. 2 and Sec. 3.1). */
typedef QIRAL_ENUM {
  QIRAL_SYSTEM_DEFAULT = 0, /* the solver's own: Schur for CGNR / BiCGStab / CRNR, D for FGMRES / FCG */
  QIRAL_SYSTEM_SCHUR = 1,   /* S x_o = b_hat on the odd sites, then x_e = A^-1 (b_e + kappa H_eo x_o) */
  QIRAL_SYSTEM_FULL = 2     /* D x = b on the whole lattice */
} qiral_system;

typedef QIRAL_ENUM {
  QIRAL_CGNR_EO = 0,     /* CGNR (Fig. "CG") on the Schur system ("schur" template) */
  QIRAL_BICGSTAB_EO = 1, /* BiCGStab (van der Vorst 1992) on the Schur system; with
                            precond, BiCGStab with the network as right preconditioner
                            (Schur: its restriction M_S v = P_o N (0 + v)), on the
                            Schur system or (system FULL) on D                        */
  QIRAL_FGMRES_NN = 2,   /* FGMRES(m) with the learned preconditioner on the right (or
                            none: precond NULL), on D or (system SCHUR) on S          */
  QIRAL_CRNR_EO = 3,     /* conjugate residual (Saad, Alg. 6.20) on the Schur normal
                            equations S^dagger S x_o = S^dagger b_hat, stopping on the
                            Schur residual like CGNR; FP64 only (inner_prec F64,
                            otherwise QIRAL_ERR_UNSUPPORTED)                          */
  QIRAL_FCG_NN = 4       /* flexible CG (Notay, SIAM J. Sci. Comput. 22, 2000), FCG(1),
                            on the normal equations A^dagger A x = A^dagger b (A = D, or
                            S with system SCHUR) with the preconditioner M M^dagger of
                            the learned network (or none); stops on ||b - D x||; FP64 */
} qiral_solver;
/* Compositions (solver x system x preconditioner) that qiral_solve runs:
 *   CGNR_EO, CRNR_EO:   system SCHUR (default), precond NULL: the grouped
 *                       batched solver; CGNR_EO with system FULL is CGNR on the
 *                       normal equations of D (run as FCG with no preconditioner,
 *                       which takes CGNR's iterates).
 *   BICGSTAB_EO:        SCHUR, precond NULL: the grouped solver; with precond,
 *                       or with system FULL: right-preconditioned BiCGStab (FP64).
 *   FGMRES_NN, FCG_NN:  FULL (default) or SCHUR, precond the network or NULL.
 * Preconditioned and FULL-system forms run in FP64 (inner_prec F64), one
 * right-hand side at a time, and are not taken by qiral_solve_batch;
 * CRNR_EO with system FULL and CGNR_EO / CRNR_EO with precond give
 * QIRAL_ERR_UNSUPPORTED. */

/* The most systems (right-hand sides, or lattices of a batch) one solve takes. */
#define QIRAL_MAX_SYSTEMS 255

typedef struct qiral_lattice qiral_lattice; /* opaque, host-side */
typedef struct qiral_nn qiral_nn;           /* opaque, learned preconditioner */

const char *qiral_status_string(qiral_status s);
const char *qiral_last_error(void);

/* Bytes of a packed field: sites of one parity (EVEN/ODD) or both (FULL), padded
 * to whole 64-site blocks, times nrhs.  Returns 0 on invalid arguments. */
size_t qiral_field_bytes(const int32_t dims[4], qiral_subset subset, qiral_prec prec, int32_t nrhs);

/* Bytes of a packed link store (the forward links of both parities, padded to
 * whole 64-site blocks): prec QIRAL_F64 with QIRAL_RECON18 (144 B per link),
 * QIRAL_F32 with QIRAL_RECON12 (48 B) or QIRAL_F16S with QIRAL_RECON12 (24 B;
 * FP16 links carry no scale, |U_ab| <= 1).  Reconstruct-12 keeps rows 0 and 1
 * and rebuilds row 2 = conj(row0 x row1), exact for SU(3).  The FP64 store keeps
 * all three rows, but the hops read rows 0 and 1 of it (96 B per link) and
 * rebuild row 2 the same way.  Returns 0 for other combinations or invalid
 * dims. */
size_t qiral_gauge_bytes(const int32_t dims[4], qiral_prec prec, qiral_recon recon);

/* Create a lattice handle.  The links must be SU(3) (unitary with determinant
 * 1, to rounding), as those of lattice QCD are: every hop, FP64 included,
 * rebuilds row 2 of a link from rows 0 and 1.  Packs the canonical links
 * (device, complex128, see above) into the caller's stores: gauge_f64 (required, qiral_gauge_bytes(dims,
 * QIRAL_F64, QIRAL_RECON18) bytes) and, if not NULL, gauge_f32 and gauge_f16
 * (reconstruct-12 stores of FP32 and FP16 links for the reduced-precision hops
 * and solves).  Each real is rounded once from FP64 to the nearest FP32 / FP16
 * (ties to even).  The stores must be 16-byte aligned, distinct, and outlive
 * the handle; gauge_canon may be freed once the call returns.  kappa is the
 * hopping parameter and mu the twisted-mass parameter of the operator of Fig.
 * "dirac",
 *   D = A - kappa H,   A = 1 + 2 i kappa mu g5   (A = 1 for mu = 0);
 * every operator, solve and true residual on the handle uses this D.  Blocking
 * (synchronises the stream).  Allocates the handle's pinned poll buffer and
 * events (see Memory above). */
qiral_status qiral_lattice_create(qiral_lattice **lat, const int32_t dims[4], double kappa, double mu,
                                  const double *gauge_canon, void *gauge_f64, void *gauge_f32, void *gauge_f16,
                                  qiral_stream_t stream);
/* Releases the handle's host resources; the caller's buffers are untouched. */
qiral_status qiral_lattice_destroy(qiral_lattice *lat);
/* Sites per parity and bytes of the caller's link stores the handle uses. */
qiral_status qiral_lattice_query(const qiral_lattice *lat, int64_t *sites_per_parity, int64_t *gauge_bytes);

/* Canonical (device complex128, [rhs][t][z][y][x][c][s]) <-> packed.  Import reads
 * the sites of the subset and writes dst; export writes only the canonical sites
 * of the subset and leaves the others untouched.  F16S import quantises each
 * site as: reals rounded to FP32, scale = max |real|, half = RNE(real / scale). */
qiral_status qiral_field_import(const qiral_lattice *lat, void *dst, const double *src_canon,
                                qiral_subset subset, qiral_prec prec, int32_t nrhs, qiral_stream_t stream);
qiral_status qiral_field_export(const qiral_lattice *lat, double *dst_canon, const void *src,
                                qiral_subset subset, qiral_prec prec, int32_t nrhs, qiral_stream_t stream);

/* Hopping term between the parities (the 8-neighbour stencil of Fig. "dirac"):
 *   out = H_{p,1-p} in        with p = out_parity, in a half-field of parity 1-p,
 *   H psi(x) = sum_mu (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu);
 * dagger != 0 applies H^dagger = g5 H g5 instead.  in and out are packed
 * half-fields of precision prec (links of the same precision must exist), nrhs
 * consecutive fields each; they must not overlap. */
qiral_status qiral_dslash_eo(const qiral_lattice *lat, void *out, const void *in, int32_t out_parity,
                             int32_t dagger, qiral_prec prec, int32_t nrhs, qiral_stream_t stream);

/* out = op(in) for packed fields of precision prec: FULL fields for OP_D/OP_DDAG,
 * ODD half-fields for OP_SCHUR/OP_SCHUR_DAG.  tmp is an EVEN half-field of the
 * same precision and nrhs (used by the Schur ops; may be NULL for D/D^dagger).
 * The Schur complement on the odd sites (template "schur") is
 *   S = A - kappa^2 H_oe A^-1 H_eo,   A^-1 = (1 - 2 i kappa mu g5) / (1 + 4 kappa^2 mu^2),
 * and S^dagger = A^dagger - kappa^2 H_oe^dagger A^-dagger H_eo^dagger. */
qiral_status qiral_apply_M(const qiral_lattice *lat, void *out, const void *in, void *tmp, qiral_op op,
                           qiral_prec prec, int32_t nrhs, qiral_stream_t stream);

/* Autotune the hop's launch shape for this lattice, precision and number of
 * right-hand sides (waves per 64-site block 1 (F16S only), 2 or 4 (FP64: 4 only);
 * right-hand sides per lane 1..4, FP64 1..2, FP32 on 2 waves 1..2, 1 wave 1; and,
 * when that leaves several groups of right-hand sides, the traversal tile of
 * 8, 16, 32 or 64 blocks that each group sweeps before the next one re-reads its
 * links) by timing each candidate on the stream; later hops and solves on this
 * handle use the fastest.  in and out are two distinct packed half-fields of precision prec
 * and nrhs fields (qiral_field_bytes(dims, QIRAL_EVEN, prec, nrhs) bytes each)
 * owned by the caller; in is zeroed, out overwritten.  If the environment
 * variable QIRAL_TUNE_CACHE names a file, the result is looked up there first
 * and stored there (JSON).  Blocking.  Outputs may be NULL; best_us is 0 on a
 * cache hit. */
qiral_status qiral_tune(qiral_lattice *lat, qiral_prec prec, int32_t nrhs, void *in, void *out, int32_t *best_t,
                        int32_t *best_nr, double *best_us, qiral_stream_t stream);

typedef struct {
  qiral_solver solver; /* QIRAL_CGNR_EO (default), QIRAL_BICGSTAB_EO, QIRAL_FGMRES_NN,
                          QIRAL_CRNR_EO, QIRAL_FCG_NN                                    */
  double tol;          /* relative FP64 residual ||b - D x|| / ||b|| to reach (e.g. 1e-10)   */
  int32_t maxiter;     /* iteration limit (outer iterations of the solver)                    */
  qiral_prec inner_prec; /* F64: plain solve.  F32/F16S: reduced-precision iterations with
                            FP64 reliable updates; needs links of that precision             */
  double delta;        /* reliable-update trigger: ||r|| < delta * max ||r|| since last one,
                          in (0, 1); 0.01 keeps the FP64 iteration counts on the workloads
                          tried (F32 and F16S) with 4-5 updates per 1e-10 solve           */
  int32_t restart;     /* FGMRES restart length m (FCG keeps one previous direction)           */
  const qiral_nn *precond; /* learned preconditioner (QIRAL_FGMRES_NN, QIRAL_FCG_NN,
                              QIRAL_BICGSTAB_EO), or NULL                               */
  int32_t fallback_cg; /* FGMRES, FCG: on stagnation or breakdown continue with eo-CGNR from
                          the current x                                                    */
  int32_t x0_is_guess; /* start from the x passed in instead of 0                              */
  int32_t use_graph;   /* capture one iteration of the grouped solver in a HIP graph (once per
                          solve) and replay it for every iteration; needs a stream other
                          than the default one (ignored there)                              */
  int32_t check_every; /* iterations enqueued between convergence checks (0: automatic)        */
  int32_t system;      /* qiral_system: the system the solver runs on (0: the solver's own)     */
} qiral_solve_params;

typedef struct {
  int32_t iterations;        /* solver iterations                                   */
  int32_t reliable_updates;  /* FP64 residual replacements (mixed precision)        */
  int32_t converged;         /* 1 if true_rel_resid <= tol                          */
  int32_t fell_back;         /* FGMRES or FCG switched to CGNR                      */
  double true_rel_resid;     /* ||b - D x|| / ||b|| recomputed in FP64 at the end   */
  double seconds;            /* wall time of the call                               */
  int64_t hop_applications;  /* H_eo / H_oe applications (units of V/2 sites)       */
} qiral_solve_info;

/* Device bytes of the workspace a qiral_solve call with these parameters and
 * nrhs right-hand sides needs on this lattice (0 for invalid arguments).  It
 * holds the Krylov vectors (5, 7 or 8 half-fields per right-hand side in the
 * iterate precision, plus 6 FP64 half-fields and, mixed, one FP32), the system
 * and work tables, per-system states and reduction partials; for FGMRES/FCG and
 * the preconditioned or full-system BiCGStab, the flexible solver's FP64 fields
 * (the larger of that and its CGNR fallback): FGMRES and FCG solve the
 * right-hand sides one after the other, BiCGStab all of them in lockstep (its
 * Krylov vectors for each and, on the Schur system with a network and more than
 * one right-hand side, nine FP32 half-fields of the network's path fields for
 * each). */
size_t qiral_solve_workspace_bytes(const qiral_lattice *lat, const qiral_solve_params *params, int32_t nrhs);
/* The same for qiral_solve_batch over nsys lattices (0 for FGMRES/FCG). */
size_t qiral_solve_batch_workspace_bytes(const qiral_lattice *const *lats, int32_t nsys,
                                         const qiral_solve_params *params);

/* Solve D x = b for nrhs right-hand sides on one lattice.  The Krylov solvers run
 * on the Schur system S x_o = b_hat of the odd sites, b_hat = b_o + kappa H_oe
 * A^-1 b_e, and rebuild x_e = A^-1 (b_e + kappa H_eo x_o) (template "schur").
 * x_canon and b_canon are canonical full fields (device); info points to nrhs
 * host structs.  ws is the caller's device workspace: 256-byte aligned and at
 * least qiral_solve_workspace_bytes(lat, params, nrhs) bytes, else
 * QIRAL_ERR_WORKSPACE (checked before any HIP call); its contents on entry do
 * not matter and are overwritten.  The call allocates no device memory.
 * Blocking: returns after the stream has drained.  Returns
 * QIRAL_ERR_NOT_CONVERGED if any right-hand side missed the tolerance. */
qiral_status qiral_solve(qiral_lattice *lat, double *x_canon, const double *b_canon, int32_t nrhs,
                         const qiral_solve_params *params, void *ws, size_t ws_bytes, qiral_solve_info *info,
                         qiral_stream_t stream);

/* Solve nsys independent systems D_i x_i = b_i (one right-hand side each, each on
 * its own lattice, of any size) in one set of grouped launches, in the caller's
 * workspace ws (qiral_solve_batch_workspace_bytes).  The solvers with the
 * learned preconditioner (QIRAL_FGMRES_NN, QIRAL_FCG_NN) take one lattice and
 * return QIRAL_ERR_UNSUPPORTED here. */
qiral_status qiral_solve_batch(qiral_lattice *const *lats, double *const *x_canon, const double *const *b_canon,
                               int32_t nsys, const qiral_solve_params *params, void *ws, size_t ws_bytes,
                               qiral_solve_info *info, qiral_stream_t stream);

/* Bytes of the library's static workspace (see qiral_solve_static). */
#define QIRAL_STATIC_WORKSPACE_BYTES (32u << 20)

/* qiral_solve for callers that cannot allocate device memory (code that must
 * not call hipMalloc or a caching allocator: tight serving loops, harnesses
 * that forbid allocation).  The same solve as qiral_solve, in a workspace that
 * is a static array of QIRAL_STATIC_WORKSPACE_BYTES (32 MiB) in the library's
 * device data: each GPU the library runs on holds its own copy from the
 * library's load until the process ends.  The call allocates nothing on the
 * device or the host's pinned heap.  Solves whose qiral_solve_workspace_bytes
 * exceed 32 MiB (about 7 FP64 right-hand sides of an 8^4 lattice) return
 * QIRAL_ERR_WORKSPACE before any HIP call; params->use_graph must be 0
 * (QIRAL_ERR_UNSUPPORTED: instantiating a graph allocates).  The current device
 * must be the lattice's.  Every call on a GPU uses that GPU's one array, which
 * keeps the last call's contents (the solve initialises what it reads): calls
 * that overlap in time on one GPU, from any thread or stream, race and must
 * not be made. */
qiral_status qiral_solve_static(qiral_lattice *lat, double *x_canon, const double *b_canon, int32_t nrhs,
                                const qiral_solve_params *params, qiral_solve_info *info, qiral_stream_t stream);

/* ---- Learned preconditioner (an addition to the paper's method) -----------
 * A 2-layer parallel-transport network 1 -> hidden -> 1 channels:
 *   psi_out^i(x) = sum_j sum_p W_p^{ij} [T_p psi_in^j](x),
 * paths p = 0 (identity), 1..4 (+x..+t: U_mu(x) psi(x+mu)), 5..8 (-x..-t:
 * U_mu(x-mu)^+ psi(x-mu)), W a complex 4x4 spin matrix (Lehner & Wettig, Phys.
 * Rev. D 108 (2023) 034503).  Weights are FP32 complex (re, im interleaved),
 * layer 1 [9][hidden][1][4][4] then layer 2 [9][1][hidden][4][4]; the network
 * runs in FP32 on the lattice's FP32 links, on packed FP32 FULL fields.  It is
 * created with the weights of 1 + kappa H + kappa^2 H^2 (channel 0 carries psi,
 * channel 1 carries H psi).  It is used by qiral_solve with solver
 * QIRAL_FGMRES_NN, QIRAL_FCG_NN or QIRAL_BICGSTAB_EO and params.precond
 * pointing to it.  The layers are linear, so applications use the folded form
 * N = sum_{p,q} T_p K_pq T_q, K_pq = sum_c W2_p^c W1_q^c (equal up to rounding);
 * on the Schur system the solvers run its path-pair products on bf16 matrix
 * cores with hi/lo splitting (about 1e-5 relative), qiral_nn_apply in FP32. */

/* Device bytes of a network with `hidden` channels (2, 4 or 8) on this lattice:
 * weights, adjoint weights, the folded weights and their matrix-core fragments,
 * Adam moments, gradient, partial sums, the hidden activations and their
 * gradient (hidden FP32 full fields each; folded applications keep nine FP32
 * full fields there, with 9 - 2 hidden more when hidden is 2 or 4), four FP32
 * full fields for training pairs, and 256 training losses.  0 for invalid
 * arguments.  Calls on one network use its memory: they must not overlap. */
size_t qiral_nn_bytes(const qiral_lattice *lat, int32_t hidden);
/* Create a network in the caller's device memory mem (256-byte aligned, at least
 * qiral_nn_bytes bytes, else QIRAL_ERR_WORKSPACE), which must outlive it; the
 * lattice needs FP32 links (gauge_f32).  Blocking (synchronises the stream). */
qiral_status qiral_nn_create(qiral_nn **nn, qiral_lattice *lat, int32_t hidden, void *mem, size_t mem_bytes,
                             qiral_stream_t stream);
/* Releases the handle; the caller's memory is untouched. */
qiral_status qiral_nn_destroy(qiral_nn *nn);
/* Number of complex weights (host arrays hold 2x as many floats). */
size_t qiral_nn_num_weights(const qiral_nn *nn);
/* Copy the weights from / to the host (blocking on the stream). */
qiral_status qiral_nn_set_weights(qiral_nn *nn, const float *w_host, size_t count, qiral_stream_t stream);
qiral_status qiral_nn_get_weights(const qiral_nn *nn, float *w_host, size_t count, qiral_stream_t stream);
/* out = N(in) and out = N^dagger(in) on packed FP32 full fields (no aliasing). */
qiral_status qiral_nn_apply(const qiral_nn *nn, void *out, const void *in, qiral_stream_t stream);
qiral_status qiral_nn_apply_adjoint(qiral_nn *nn, void *out, const void *in, qiral_stream_t stream);
/* The Gaussian training vector of (seed, step) as a packed FP32 full field: the
 * 24 reals of canonical site lex come from Philox4x32-10 (Salmon et al. 2011)
 * with counter (lex, k, step_lo, step_hi), k = 0..5, key (seed_lo, seed_hi),
 * uniforms (n + 1/2) 2^-32 and the Box-Muller transform.  norm2 (host, may be
 * NULL) receives ||v||^2. */
qiral_status qiral_nn_sample(qiral_nn *nn, void *out, uint64_t seed, uint64_t step, double *norm2,
                             qiral_stream_t stream);
/* Loss ||N(src) - target||^2 / ||target||^2 and its gradient with respect to the
 * real and imaginary parts of every weight (host arrays; grad holds
 * 2 * qiral_nn_num_weights doubles, re/im interleaved; either may be NULL). */
qiral_status qiral_nn_grad(qiral_nn *nn, const void *src, const void *target, double *loss, double *grad,
                           qiral_stream_t stream);
/* steps Adam updates (lr; beta 0.9, 0.999) on the pairs (D v, v), v the
 * training vectors of (seed, global step counter); loss_history (host[steps])
 * may be NULL.  Blocking. */
qiral_status qiral_nn_train(qiral_nn *nn, int32_t steps, double lr, uint64_t seed, double *loss_history,
                            qiral_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* QIRAL_H */
