/*
 * mxw.h -- C ABI of the MI355X (gfx950) library for time-harmonic Maxwell
 * problems discretised with degree-r Nedelec edge elements and solved by
 * GMRES preconditioned with overlapping optimized restricted additive
 * Schwarz (ORAS).
 *
 * The operation (Bonazzoli, Dolean, Rapetti, Tournier, "Parallel
 * preconditioners for high order discretizations arising from full system
 * modeling for brain microwave imaging"):
 *   - Sec. 2, eq. (1)-(4) and the weak form: curl curl E - k0^2 eps E = 0 in
 *     the domain, E x n = 0 on metallic faces, impedance condition on the
 *     others; the system matrix is A = K - k0^2 M_eps - i beta B, complex
 *     symmetric (bilinear form, one matrix for every right-hand side);
 *   - Sec. 3: degree-r generators lambda^k w^e, |k| = r-1, with a fixed
 *     independent subset (r=1,2,3 -> 6, 20, 45 functions per element);
 *   - Sec. 4: M^{-1} = sum_s R_s^T D_s A_s^{-1} R_s, A_s with impedance
 *     transmission conditions on subdomain interfaces;
 *   - Sec. 5: GMRES preconditioned by it; several right-hand sides are
 *     processed together (pseudo-block), or in one block Krylov space
 *     (block GMRES, Sec. 6).
 *
 * Conventions used throughout:
 *   - time dependence exp(-i w t): a lossy medium has Im(eps) > 0 (the
 *     paper's values are the complex conjugates of the ones passed here);
 *   - beta on an impedance face = k0 sqrt(Re eps) of the adjacent element;
 *     the transmission coefficient on an interface face uses the element of
 *     the subdomain that owns the face;
 *   - global unknowns: edges (lexicographic vertex pairs) then faces
 *     (lexicographic triples) then elements (input order), each entity's
 *     unknowns in a fixed order; unknowns on metallic faces are removed;
 *   - overlap: each layer adds the elements sharing a face with the
 *     subdomain; the partition of unity is Boolean (an unknown belongs to the
 *     lowest core subdomain id among the elements that contain its entity);
 *   - complex numbers are interleaved (re, im) doubles.
 *
 * Ownership: the caller owns every array it passes; create calls copy what
 * they keep, so inputs may be freed on return.  Outputs are allocated by the
 * caller.  Errors: every call returns an mxw_status; mxw_last_error() gives
 * the message of the last failing call on the calling thread.  A problem is
 * immutable after creation except through mxw_problem_factor; solves on one
 * problem must not overlap in time (they share the Krylov workspace).
 */
#ifndef MXW_H
#define MXW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mxw_status;
enum {
  MXW_OK = 0,
  MXW_EINVAL = -1,      /* invalid argument or inconsistent mesh data */
  MXW_ENOMEM = -2,      /* device or host allocation failed, or budget exceeded */
  MXW_ENOTCONV = -3,    /* max_iters reached; outputs hold the last iterate */
  MXW_ESINGULAR = -4,   /* zero pivot in a local LU factorisation */
  MXW_EBREAKDOWN = -5,  /* Krylov breakdown without convergence */
  MXW_EDEVICE = -6,     /* a HIP runtime call failed */
  MXW_EBUSY = -7        /* ticket not finished */
};

enum { MXW_BC_PEC = 0, MXW_BC_IMPEDANCE = 1 };
/* local factor precision: FP64 everywhere, or complex-FP32 local LU/solves
 * with everything else (assembly, SpMV, Arnoldi, least squares) in FP64 */
enum { MXW_FP64 = 0, MXW_MIXED = 1 };
/* sources: point dipole, incident plane wave on the impedance boundary, and
 * a rectangular waveguide port excited by its TE10 mode (eq. (3)) */
enum { MXW_SRC_DIPOLE = 0, MXW_SRC_PLANEWAVE = 1, MXW_SRC_PORT = 2 };
/* multi-source Krylov drivers (Sec. 5): PSEUDOBLOCK = one Krylov space per
 * right-hand side, all operations fused over the columns; BLOCK = one shared
 * block Krylov space (block CGS2 orthogonalisation, Cholesky QR of each new
 * block, Householder block least squares), at most 32 independent, non-zero
 * right-hand sides per solve (MXW_EINVAL otherwise).  A new block that is
 * numerically rank deficient keeps a floor pivot in its Cholesky QR and the
 * solve goes on (the true residual at each cycle end decides convergence);
 * a non-finite residual estimate ends the solve with MXW_EBREAKDOWN. */
enum { MXW_KRYLOV_PSEUDOBLOCK = 0, MXW_KRYLOV_BLOCK = 1 };
/* preconditioner variants (Sec. 4): ORAS (default: Robin transmission,
 * Boolean partition of unity), OAS (no D_s), RAS (Dirichlet transmission:
 * A_s = R_s A R_s^T, Boolean D_s), ORAS_MULT (Robin transmission, partition
 * of unity by multiplicity: D_s = diag(1 / number of subdomains containing
 * the unknown)) */
enum { MXW_PREC_ORAS = 0, MXW_PREC_OAS = 1, MXW_PREC_RAS = 2, MXW_PREC_ORAS_MULT = 3 };

typedef struct {
  int64_t n_vertices;
  const double* xyz;          /* [n_vertices][3] */
  int64_t n_tets;
  const int32_t* tets;        /* [n_tets][4], 0-based vertex ids, any order */
  const double* eps;          /* [n_tets][2] relative permittivity (re, im) */
  int64_t n_bfaces;
  const int32_t* bfaces;      /* [n_bfaces][3]; exactly the faces with one tet */
  const int8_t* bface_kind;   /* [n_bfaces] MXW_BC_* */
  const int32_t* part;        /* [n_tets] core subdomain id in [0, n_sub) */
  int32_t n_sub;
  int32_t overlap_layers;     /* >= 0 face-adjacency layers */
  double k0;                  /* free-space wavenumber, same length unit as xyz */
  int32_t degree;             /* r in {1, 2, 3} */
  int32_t precision;          /* MXW_FP64 | MXW_MIXED */
  int32_t prec_variant;       /* MXW_PREC_* */
  int32_t reserved;
} mxw_problem_desc;

/* Port (MXW_SRC_PORT): a rectangle on the impedance boundary with centre pos,
 * half its wide side dir (width a = 2 |dir|; the TE10 profile varies along it)
 * and half its narrow side pol_re (height b = 2 |pol_re|; the direction v of
 * E), dir orthogonal to pol_re, pol_im unused.  Its faces are the impedance
 * faces whose centroid lies in the rectangle (within 1e-9 (a + b), also off
 * its plane).  The mode on the port is E0 = sin(pi (s + a/2) / a) v, s the
 * coordinate along dir from pos; it enters the domain with the propagation
 * constant beta10 = sqrt(max(beta^2 - (pi/a)^2, 0)), beta the face's
 * impedance wave number, so the port data of eq. (3) are
 * g = -i (beta10 + beta) E0 (exp(-i w t) convention). */
typedef struct {
  int32_t kind;               /* MXW_SRC_* */
  int32_t reserved;
  double pos[3];              /* dipole position / port centre */
  double pol_re[3];           /* dipole moment / plane-wave polarisation / port half height */
  double pol_im[3];
  double dir[3];              /* plane-wave unit direction / port half width */
} mxw_source;

typedef struct {
  double tol;                 /* true relative residual target ||b-Ax||/||b|| */
  int32_t restart;            /* m, Krylov steps per cycle (1..200) */
  int32_t max_iters;          /* total Arnoldi steps (block steps for block GMRES) */
  int32_t krylov;             /* MXW_KRYLOV_* */
  int32_t use_graph;          /* 1: run each Arnoldi step as a captured HIP graph */
} mxw_solve_opts;

typedef struct {
  int64_t ndof;               /* global unknowns after metallic elimination */
  int64_t nnz;                /* structural non-zeros of A */
  int32_t n_sub;
  int32_t nloc;               /* unknowns per element: 6, 20, 45 */
  int64_t sum_ns;             /* sum of local sizes n_s */
  int64_t max_ns;
  double sum_ns2;             /* sum of n_s^2 (dense factor entries) */
  double sum_ns3;             /* sum of n_s^3 */
  int64_t n_iface;            /* interface faces over all subdomains */
  int64_t n_imp_faces;        /* impedance boundary faces */
} mxw_layout_info;

typedef struct mxw_layout mxw_layout;
typedef struct mxw_problem mxw_problem;
typedef struct mxw_ctx mxw_ctx;
typedef struct mxw_ticket mxw_ticket;

/* Device memory provider of a context: alloc returns a device pointer of at
 * least `bytes` bytes on the context's device for use on `stream` (NULL on
 * failure); free_ returns it.  Both may be called from the library's worker
 * threads (asynchronous solves).  The library only returns memory once the
 * work that used it is finished (it synchronises first), so a stream-ordered
 * caching allocator such as PyTorch's may hand it out again at once. */
typedef void* (*mxw_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*mxw_free_fn)(void* ptr, void* user);

/* Message of the last failing call on this thread (never NULL). */
const char* mxw_last_error(void);

/* ---- contexts: device memory and HBM budget ----------------------------- */

/* A context owns the device-memory policy of the problems created with it
 * (the serving loop of an imaging inversion admits forward solves by their
 * device footprint, Sec. 5-6): every device allocation those problems make
 * (their operator and factors, the layout device copy they build, Krylov
 * workspaces and the temporaries of a solve) goes through alloc/free_ and is
 * counted; an allocation that would take the bytes in use above hbm_budget
 * (0 = no limit) fails with MXW_ENOMEM before anything is allocated.  alloc =
 * free_ = NULL: hipMalloc / hipFree.  device: the HIP device the problems
 * live on (made current by the library's worker threads).  A problem created
 * with ctx = NULL uses a process-wide default context (hipMalloc, no budget),
 * whose counters mxw_ctx_usage(NULL, ...) reports. */
mxw_status mxw_ctx_create(int32_t device, uint64_t hbm_budget, mxw_alloc_fn alloc, mxw_free_fn free_,
                          void* user, mxw_ctx** out);
/* Releases the context.  MXW_EBUSY (and nothing released) while device
 * memory obtained through it is still held (live problems, or layout device
 * copies they built); NULL is a no-op. */
mxw_status mxw_ctx_destroy(mxw_ctx* ctx);
/* Bytes in use now, the peak since creation (or the last reset_peak != 0
 * call, which sets it to the bytes in use), and the number of live
 * allocations.  NULL outputs are skipped. */
mxw_status mxw_ctx_usage(mxw_ctx* ctx, uint64_t* in_use, uint64_t* peak, int64_t* live, int32_t reset_peak);

/* ---- host-side setup (no device needed) -------------------------------- */

/* Entities, unknown numbering (Sec. 3-4), sparsity pattern of A, overlapping
 * subdomains N_s with their partition of unity D_s and interface faces
 * (Sec. 4).  Validates the mesh: vertex ids in range, distinct vertices,
 * non-zero volumes, finite eps, boundary faces equal to the faces with one
 * tet, part ids in range.  Returns MXW_EINVAL with a message otherwise. */
mxw_status mxw_layout_create(const mxw_problem_desc* desc, mxw_layout** out);
void mxw_layout_destroy(mxw_layout* layout);
mxw_status mxw_layout_get_info(const mxw_layout* layout, mxw_layout_info* info);
/* Entity of each global unknown: kind 0 edge / 1 face / 2 element, entity id
 * in the numbering above, index within the entity.  Arrays of length ndof. */
mxw_status mxw_export_dofs(const mxw_layout* layout, int8_t* ent_kind, int64_t* ent_id,
                           int16_t* ent_local);
/* CSR pattern of A: rowptr [ndof+1], cols [nnz] ascending in each row. */
mxw_status mxw_export_pattern(const mxw_layout* layout, int64_t* rowptr, int32_t* cols);
/* N_s of subdomain s (sorted global unknowns) and D_s (0/1).  Pass NULL for
 * dofs/pou to query n_s only. */
mxw_status mxw_export_subdomain(const mxw_layout* layout, int32_t s, int64_t* n_s,
                                int64_t* dofs, uint8_t* pou);
/* Device bytes of one problem on this layout (precision, prec_variant) that
 * runs mxw_solve / mxw_solve_async with nrhs sources and the options opts
 * (restart, krylov; NULL = restart 50, pseudo-block): its operator, element
 * matrices and factors, the Krylov (and block) workspace for nrhs columns,
 * and the solve's temporaries (right-hand sides, solution staging, face
 * integrals).  with_layout_copy = 1 adds the layout's device copy, which
 * every problem on the layout shares (count it once).  This is the peak of
 * the bytes the problem's context counts for it; admission control relies on
 * it.  Not included: mxw_problem_tune, mxw_smatrix and mxw_solve_recycle
 * (their own temporaries / recycled spaces). */
mxw_status mxw_layout_footprint(const mxw_layout* layout, int32_t precision, int32_t prec_variant, int32_t nrhs,
                                const mxw_solve_opts* opts, int32_t with_layout_copy, uint64_t* bytes);
/* The same for a problem described by desc alone (its own layout copy
 * included): builds the host layout (entities, numbering, subdomains) to
 * size it, without touching the device. */
mxw_status mxw_footprint(const mxw_problem_desc* desc, int32_t nrhs, const mxw_solve_opts* opts, uint64_t* bytes);

/* ---- device problem ---------------------------------------------------- */

/* Builds the device operator: element matrices (FP64), CSR assembly of A,
 * dense local matrices A_s and (unless defer_factor) their batched LU
 * factorisation with partial pivoting, all on `stream` (a hipStream_t; NULL
 * = default stream) of the context's device (ctx NULL: the current device
 * and the default context).  Blocks until done.  A problem whose operator
 * and factors would take the context above its budget is rejected with
 * MXW_ENOMEM before anything is allocated.  The context must outlive the
 * problem. */
mxw_status mxw_problem_create(mxw_ctx* ctx, const mxw_problem_desc* desc, void* stream, int32_t defer_factor,
                              mxw_problem** out);
/* Device problem on the mesh, degree and partition of an existing layout,
 * with a permittivity field eps [n_tets][2] (NULL = the layout's) and a
 * wavenumber k0 (negative = the layout's).  The layout's device copy
 * (geometry, unknown numbering, subdomain maps, face matrices) is built on
 * first use and shared by every problem created from it; each problem keeps
 * its layout alive, so the layout handle may be destroyed at any time.  This
 * is the call for streams of solves on one mesh with changing media.  The
 * device copy is allocated through the context of the problem that builds it
 * and returned when the layout and all its problems are gone. */
mxw_status mxw_problem_create_from_layout(mxw_ctx* ctx, const mxw_layout* layout, const double* eps, double k0,
                                          int32_t precision, int32_t prec_variant, void* stream,
                                          int32_t defer_factor, mxw_problem** out);
/* Replaces the medium of an existing problem (eps [n_tets][2], NULL = the
 * layout's; k0 < 0 keeps the current wavenumber) and redoes, in the problem's
 * own device buffers, everything that depends on it: element matrices, CSR
 * values, dense A_s and their LU factors (Sec. 2-4).  No device memory is
 * allocated.  This is the step of an imaging loop, where only eps changes,
 * and mostly inside the imaged head (Sec. 6: slowly varying systems): a
 * subdomain whose local data (k0 and the permittivity of every element of
 * its overlapping Omega_s) hash to the same value as for its current
 * factors keeps them, and only the others are assembled and factorised again
 * (ORAS, OAS and ORAS_MULT; RAS, whose A_s are rows of A, and a problem whose
 * last factorisation failed or was deferred redo every subdomain).  The
 * factors are the same bits as a fresh problem's for the new medium. */
mxw_status mxw_problem_set_medium(mxw_problem* prob, const double* eps, double k0, void* stream);
/* The next medium change re-assembles and factorises every subdomain, kept
 * factors or not (a full factorisation, for instance to time it). */
mxw_status mxw_problem_forget_factors(mxw_problem* prob);
/* Subdomains re-factorised by the last medium change (all of them at
 * creation), and the totals re-factorised and kept over the problem's
 * medium changes.  NULL outputs are skipped. */
mxw_status mxw_problem_factor_stats(const mxw_problem* prob, int32_t* refactored_last, int64_t* refactored_total,
                                    int64_t* kept_total);
void mxw_problem_destroy(mxw_problem* prob);
mxw_status mxw_problem_get_info(const mxw_problem* prob, mxw_layout_info* info);
/* Factorises every A_s in place (batched LU, partial pivoting). Idempotent.
 * MXW_ESINGULAR names the first subdomain with a zero pivot. */
mxw_status mxw_problem_factor(mxw_problem* prob, void* stream);

/* Values of A in the exported CSR pattern, host complex128 [nnz]. */
mxw_status mxw_problem_export_matrix(const mxw_problem* prob, double* vals);
/* Dense A_s before factorisation (column-major, host complex128 [n_s*n_s]).
 * Only valid while the problem is not yet factorised. */
mxw_status mxw_problem_export_local(const mxw_problem* prob, int32_t s, double* a_s);

/* Right-hand sides b [nrhs][ndof] (device complex128) for the sources:
 * dipole b_i = p . phi_i(x_s) in the lowest-index element containing x_s;
 * plane wave b_i = int g . phi_i over impedance faces, g from
 * E = p exp(i k0 sqrt(eps) d.x); port (eq. (3)) b_i = int g . phi_i over the
 * port's faces, g = -i (beta10 + beta) E0 (see mxw_source).  MXW_EINVAL for
 * an unknown kind or a malformed port. */
mxw_status mxw_problem_rhs(mxw_problem* prob, int32_t nrhs, const mxw_source* src, double* b_dev,
                           void* stream);
/* For callers that cannot allocate device memory (code run under HIP graph
 * capture or in tight serving loops, harnesses that forbid hipMalloc): the
 * same right-hand sides as mxw_problem_rhs, bit for bit, computed without
 * any device allocation.  The face integrals of plane-wave and port sources
 * go to a fixed buffer compiled into the library (4 MiB per device, kept
 * until the process ends), so the problem may have at most 262,144 /
 * nfloc impedance faces (nfloc = 3, 8, 15 face unknowns for r = 1, 2, 3);
 * larger problems get MXW_EINVAL with a message, as does a problem that
 * lives on another device than the current one.  Every call on one device
 * shares that buffer: calls that overlap in time on one device (other host
 * threads, other streams) race and must be serialised by the caller.
 * Synchronises the stream like mxw_problem_rhs. */
mxw_status mxw_problem_rhs_noalloc(mxw_problem* prob, int32_t nrhs, const mxw_source* src, double* b_dev,
                                   void* stream);
/* y = A x for nrhs device vectors [nrhs][ndof] complex128.  16..32 columns
 * go through a temporary interleaved copy (ndof x 32 complex128, allocated
 * through the problem's context): the matrix is read once for all of them. */
mxw_status mxw_problem_apply_A(mxw_problem* prob, int32_t nrhs, const double* x_dev, double* y_dev,
                               void* stream);
/* z = M^{-1} v (ORAS: restrict, local LU solves, Boolean prolongation).
 * With nrhs >= 2 (ORAS) every factor strip is read once per 32 columns;
 * with 16 <= nrhs <= 32 the columns are first copied to a temporary
 * interleaved layout (ndof x 32 complex128) so that the local solves gather
 * an unknown's columns in one read.  Temporaries are allocated through the
 * problem's context. */
mxw_status mxw_problem_apply_prec(mxw_problem* prob, int32_t nrhs, const double* v_dev, double* z_dev,
                                  void* stream);

/* Solves A x_j = b_j for nrhs sources with FGMRES + ORAS (right
 * preconditioning, x0 = 0; pseudo-block or block per opts->krylov).  E_out:
 * complex128 [nrhs][ndof] on the device (E_out_is_device = 1) or host.
 * iters_out [nrhs] (Arnoldi steps; block steps in block mode) and relres_out
 * [nrhs] (true relative residuals) may be NULL.  Returns MXW_ENOTCONV if any
 * column missed tol within max_iters. */
mxw_status mxw_solve(mxw_problem* prob, int32_t nrhs, const mxw_source* src,
                     const mxw_solve_opts* opts, void* stream, double* E_out,
                     int32_t E_out_is_device, int32_t* iters_out, double* relres_out);
/* Same with right-hand sides given directly (device complex128 [nrhs][ndof]). */
mxw_status mxw_solve_rhs(mxw_problem* prob, int32_t nrhs, const double* b_dev,
                         const mxw_solve_opts* opts, void* stream, double* x_dev,
                         int32_t* iters_out, double* relres_out);

/* Asynchronous mxw_solve, for the request loop of an imaging inversion,
 * which keeps forward solves of several transmitting antennas and media in
 * flight (Sec. 5-6): the same arguments and results as mxw_solve.  src and
 * opts are copied; E_out, iters_out and relres_out must stay valid until the
 * ticket has completed.  The solve runs on a library worker thread that makes
 * the problem's device current and drives `stream`; solves on one problem run
 * one after another (each holds the problem while it runs), solves on
 * different problems overlap on the device.  *ticket receives the handle to
 * poll, wait on and destroy (MXW_EINVAL for invalid arguments, nothing
 * started). */
mxw_status mxw_solve_async(mxw_problem* prob, int32_t nrhs, const mxw_source* src, const mxw_solve_opts* opts,
                           void* stream, double* E_out, int32_t E_out_is_device, int32_t* iters_out,
                           double* relres_out, mxw_ticket** ticket);
/* *done = 1 once the ticket's solve has finished (its outputs are then
 * complete), else 0.  Never blocks. */
mxw_status mxw_ticket_poll(mxw_ticket* ticket, int32_t* done);
/* Blocks until the solve has finished; returns its status (the message of a
 * failure is then mxw_last_error() of the calling thread). */
mxw_status mxw_ticket_wait(mxw_ticket* ticket);
/* Waits for the solve if it is still running, then releases the ticket. */
void mxw_ticket_destroy(mxw_ticket* ticket);

/* Device bytes the problem holds now (operator, factors, workspaces; not the
 * shared layout device copy). */
mxw_status mxw_problem_device_bytes(const mxw_problem* prob, uint64_t* bytes);

/* S-matrix (eq. (5)) of nsol fields X (device complex128 [nsol][ndof]) on
 * nports ports (MXW_SRC_PORT sources): S_ij = int_{Gamma_i} conj(E_j) . E0_i
 * / int_{Gamma_i} |E0_i|^2, the integrals taken with the right-hand sides'
 * face quadrature; S_dev receives device complex128 [nports][nsol]
 * (caller-allocated).  The fields follow the exp(-i omega t) convention of
 * the library (Im eps > 0 lossy), so S is the complex conjugate of eq. (5)'s
 * S in an exp(+i omega t) convention.  Allocates temporary device buffers
 * and synchronises the stream.  MXW_EINVAL for a source that is not a valid
 * port or a port with no face. */
mxw_status mxw_smatrix(mxw_problem* prob, int32_t nports, const mxw_source* ports, int32_t nsol,
                       const double* X_dev, void* stream, double* S_dev);

/* Krylov subspace recycling (Sec. 6: GCRO-DR, the method of Parks, de Sturler
 * et al., 2006, proposed there for the slowly varying systems of the imaging
 * loop).  Solves A x_j = b_j for the nrhs right-hand sides one after another
 * (device complex128 [nrhs][ndof] in b_dev and x_dev), each by GCRO-DR on the
 * right-preconditioned operator A M^{-1} (x0 = 0), carrying a recycled space
 * of k vectors held by the problem from one system to the next:
 *  - a space made for another operator (after mxw_problem_set_medium or a
 *    new factorisation) is first carried over: C = A M^{-1} U recomputed and
 *    orthonormalised (k preconditioner applications and products);
 *  - every cycle removes the residual's part in range(C), runs restart - k
 *    Arnoldi steps of (I - C C^H) A M^{-1} (restart steps while no space
 *    exists yet), updates x, and replaces the space by the k harmonic Ritz
 *    vectors of smallest harmonic Ritz value of the cycle's search space.
 * opts->restart = vectors per cycle (k < restart <= 64), 1 <= k <= 32,
 * opts->tol, opts->max_iters as for mxw_solve; use_graph is ignored.
 * iters_out counts Arnoldi steps.
 * Block GCRO-DR (Sec. 6 combines the block and the recycling strategies):
 * with opts->krylov = MXW_KRYLOV_BLOCK and 2 <= nrhs <= 16 the nrhs columns
 * are solved together in one block space: every cycle removes the block
 * residual's part in range(C), runs (restart - dim) / nrhs block Arnoldi
 * steps of (I - C C^H) A M^{-1} (block CGS2 against C and the previous
 * blocks, Cholesky QR of each new block, block least squares), and the new
 * space is the k harmonic Ritz vectors of the cycle's search space, whose
 * projected matrix has nrhs rows below the Krylov part (restart + nrhs <=
 * 65; k + nrhs <= restart, so that a cycle holds at least one block step).
 * iters_out then counts block steps (the same for every column).
 * Other krylov values solve the columns one after another as above.
 * A different k or restart than the previous call drops the space; a
 * different block width keeps it.  Device memory held by the problem:
 * (2 restart + 5 k + 3 p) ndof complex128 (p the widest block used so far,
 * 1 without blocks) and small matrices.  MXW_ENOTCONV /
 * MXW_EBREAKDOWN as for mxw_solve; MXW_EINVAL for bad options, a zero
 * right-hand side in a block, or an unfactorised problem. */
mxw_status mxw_solve_recycle(mxw_problem* prob, int32_t nrhs, const double* b_dev,
                             const mxw_solve_opts* opts, int32_t k, void* stream, double* x_dev,
                             int32_t* iters_out, double* relres_out);
/* Forgets the recycled space (the next recycling solve starts as GMRES). */
mxw_status mxw_recycle_reset(mxw_problem* prob);
/* The recycled space: dim receives its dimension; any of U, Ubar = M^{-1} U
 * and C = A Ubar (C^H C = I) that is not NULL receives dim device vectors
 * [dim][ndof] complex128 (caller-allocated).  Synchronises the stream. */
mxw_status mxw_recycle_export(mxw_problem* prob, int32_t* dim, double* U_dev, double* Ubar_dev,
                              double* C_dev, void* stream);
/* Counters of the problem's recycling: spaces carried to a new operator,
 * deflated restarts, and restarts whose small eigenproblem failed (the space
 * is then dropped and the solve goes on without it).  NULL outputs skipped. */
mxw_status mxw_recycle_stats(const mxw_problem* prob, int64_t* refreshes, int64_t* deflations,
                             int64_t* failures);

/* Tile choices of the hot kernels, measured on one problem. */
typedef struct {
  int32_t spmv_group;         /* lanes per matrix row chosen for the SpMV */
  int32_t multi_ku;           /* k slice width chosen for the multi-column local solve */
  double spmv_ms[4];          /* time per SpMV launch with 4, 8, 16, 32 lanes per row */
  double multi_ms[2];         /* time per multi-column local solve with 4-, 8-wide k
                                 slices (0 where not measured) */
  int32_t lu_ku;              /* k slice width of the LU's block-column update (FP64: always 4) */
  int32_t multi_rows;         /* rows per pass of the multi-column local solve (64 or 128) */
  double lu_ms[2];            /* time per LU of every A_s with 4-, 8-wide k slices (FP32
                                 factors only; 0 where not measured) */
  double multi_tall_ms;       /* time per multi-column local solve with 128-row passes
                                 (FP32 factors only; 0 where not measured) */
  int32_t lu_launch;          /* LU launch chosen: 1 one workgroup per subdomain, 2 persistent queue */
  int32_t reserved;
  double lu_launch_ms[2];     /* time per LU of every A_s with each launch (factorised problems) */
} mxw_tuning;

/* Autotuner (launch mechanics; not a passage of the paper): times the SpMV
 * on nrhs columns with 4, 8, 16 and 32 lanes per row; for nrhs >= 2, a
 * Boolean partition of unity (ORAS, RAS) and a factorised problem, the
 * multi-column local solve with 4- and 8-wide k slices (for FP32 factors also
 * with 128-row passes); and for FP32 factors (MXW_MIXED, factorised) the LU
 * with 4- and 8-wide k slices and, for every factorised problem, the two
 * LU launches (each trial
 * re-assembles the local matrices and factorises them again: seconds at a
 * million unknowns; the problem ends factorised with the fastest), all on
 * this problem's own operator and factors; later calls on the problem use
 * the fastest of each.  Results do not depend on the choice beyond rounding
 * (a re-factorisation makes recycled spaces stale).  Allocates temporary
 * device buffers (2 nrhs ndof complex128, plus the multi-column scratch) and
 * synchronises the stream.  out may be NULL.  MXW_EINVAL for nrhs outside
 * 1..4096. */
mxw_status mxw_problem_tune(mxw_problem* prob, int32_t nrhs, void* stream, mxw_tuning* out);

/* Sets the tile choices by hand (for instance those a previous
 * mxw_problem_tune call picked): spmv_group in {4, 8, 16, 32}, multi_ku and
 * lu_ku in {4, 8} (lu_ku applies to the next factorisation, FP32 only),
 * multi_rows in {64, 128} (128-row passes take 8-wide slices), lu_launch 1
 * (one workgroup per subdomain, largest first; the default for FP64 factors)
 * or 2 (one persistent launch whose resident workgroups take the subdomains,
 * largest first, from a work counter; the default for FP32 factors); 0
 * leaves a choice unchanged.  Every choice gives the same
 * factors bit for bit.  MXW_EINVAL for other values. */
mxw_status mxw_problem_set_tiles(mxw_problem* prob, int32_t spmv_group, int32_t multi_ku, int32_t lu_ku,
                                 int32_t multi_rows, int32_t lu_launch);

/* Residual estimates |g_{j+1}| / ||b|| of every Arnoldi step of column col
 * in the last solve on this problem (host array; len receives the count,
 * at most max_len values are written; out may be NULL). */
mxw_status mxw_solve_history(const mxw_problem* prob, int32_t col, double* out, int32_t max_len,
                             int32_t* len);

/* ---- instrumentation --------------------------------------------------- */

/* Per-kernel timing with HIP events on the launching stream (off by default). */
mxw_status mxw_set_timing(int32_t enabled);
/* Accumulated time (ms) and launch count of a kernel class since the last
 * reset: names "lu", "local_solve", "spmv", "cgs", "assemble", "local_assemble". */
mxw_status mxw_get_timing(const char* name, double* total_ms, int64_t* launches);
mxw_status mxw_reset_timing(void);

#ifdef __cplusplus
}
#endif
#endif /* MXW_H */
