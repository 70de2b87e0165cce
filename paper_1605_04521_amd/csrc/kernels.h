// Kernel launchers (host-callable) of the mxw library.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mxw_internal.h"

namespace mxw {

constexpr int kLuNB = 32;   // LU panel width = block size of the triangular sweeps

// Start/stop events for the next timed launch, if kernel timing is on.
bool take_timer_events(hipEvent_t* a, hipEvent_t* b);

// Launch through hipExtLaunchKernelGGL when timing events are pending.
template <typename F, typename... Args>
inline void timed_launch(F kernel, dim3 grid, dim3 block, unsigned shmem, hipStream_t st, Args... args) {
  hipEvent_t a, b;
  if (take_timer_events(&a, &b))
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, a, b, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
}

void launch_element(hipStream_t st, int64_t nt, const double* xyz, const int* tets, const double* eps,
                    const Term* phi, const Term* curl, int nloc, int ncurl, double k0sq, double2* AT);
void launch_face(hipStream_t st, int64_t nft, const double* xyz, const int* fvert, const Term* fphi, int nfloc,
                 double* BF);

struct AssembleArgs {
  int64_t ndof;
  const int64_t* rowptr;
  const int* cols;
  const int* dof_ent;
  const int64_t* ent_tet_ptr;
  const int* ent_tets;
  const int64_t* ent_imp_ptr;
  const int* ent_imps;
  const int* tet_dofs;
  int nloc;
  const double2* AT;
  const int* imp_ft;
  const double* imp_beta;
  const int* ft_dofs;
  int nfloc;
  const double* BF;
  double2* vals;
};
void launch_assemble_rows(hipStream_t st, const AssembleArgs& a);

struct LocalAssembleArgs {
  int n_sub;
  const int64_t* foff;
  const int* nsz;
  const int* lds;
  const int64_t* tet_ptr;
  const int* tets;
  const int* lmap;
  const double2* AT;
  int nloc;
  const int64_t* face_ptr;
  const int* face_ft;
  const double* face_coef;
  const int* face_lmap;
  const double* BF;
  int nfloc;
  const int* list = nullptr;   // subdomains to assemble (n_sub of them); nullptr = 0 .. n_sub-1
};
template <typename R>
void launch_assemble_local(hipStream_t st, const LocalAssembleArgs& a, R* F);
template <typename R>
void launch_local_from_csr(hipStream_t st, int n_sub, R* F, const int64_t* foff, const int* nsz, const int* lds,
                           const int64_t* poff, const int* sub_dofs, const int64_t* rowptr, const int* cols,
                           const double2* vals);

void launch_rhs_dipole(hipStream_t st, const double* xyz, const int* tets, const int* tet_dofs, const Term* phi,
                       int nloc, int64_t t, const double lam[4], const double pr[3], const double pi[3],
                       double2* b);

struct PlaneWaveArgs {
  int nimp;
  int64_t ndof;
  const double* xyz;
  const int* fvert;
  const int* imp_ft;
  const int* imp_opp;
  const double* imp_beta;
  const double* imp_eps;
  const Term* fphi;
  int nfloc;
  double k0;
  int nq;
  const double* gx;
  const double* gw;
  const int* dof_ent;
  const int64_t* ent_imp_ptr;
  const int* ent_imps;
  const int* ft_dofs;
};
void launch_rhs_planewave(hipStream_t st, const PlaneWaveArgs& a, const double pr[3], const double pi[3],
                          const double d[3], double2* work, double2* b);
// rectangular TE10 port: mode 0 excitation g (eq. (3)), mode 1 mode weights
// and, in den, the mode's squared norm on the port (eq. (5)); the face
// integrals are added into b
void launch_rhs_port(hipStream_t st, const PlaneWaveArgs& a, const double c[3], const double u[3], const double v[3],
                     double aw, double bh, int mode, double2* work, double* fnorm, double* den, double2* b);
void launch_smatrix_finish(hipStream_t st, int nsol, int np, const double2* num, const double* den, double2* S);

// queue != nullptr: persistent launch (a resident grid takes the n_sub
// subdomains of order from a counter at *queue, which the launch resets)
template <typename R>
void launch_lu(hipStream_t st, int n_sub, R* F, const int64_t* foff, const int* nsz, const int* lds, int* perm,
               const int64_t* poff, R* scratch, int* info, const int* order, int ku, int* queue = nullptr);

struct LocalSolveArgs {
  int n_sub;
  int max_ns;
  const int64_t* foff;
  const int* nsz;
  const int* lds;
  const int* perm;
  const int64_t* poff;
  const int* sub_dofs;
  const uint8_t* pou;
  const int* order;
  // optional interleaved copy of the input ([ndof][interleaved_cols()],
  // zero-padded columns): the multi-column solves gather a row's columns as
  // one contiguous read (at most interleaved_cols() columns)
  const double2* vil = nullptr;
};
template <typename R>
void launch_local_solve(hipStream_t st, const LocalSolveArgs& a, const R* F, const double2* v, int64_t vstride,
                        double2* z, int64_t zstride, double2* ys, int64_t ystride, int ncol, const int* active);
hipError_t prepare_local_solve(size_t dyn_bytes_double, size_t dyn_bytes_float);
// all columns at once: factor strips read once per chunk of multi_chunk_cols() columns
template <typename R>
void launch_local_solve_multi(hipStream_t st, const LocalSolveArgs& a, const R* F, const double2* v, int64_t vstride,
                              double2* z, int64_t zstride, R* xbuf, int64_t sum_ns, int ncol, const int* active,
                              int ku, int rows);
int multi_chunk_cols();
void launch_gather_all(hipStream_t st, int64_t ndof, const int64_t* ptr, const int64_t* pos, const double2* ys,
                       int64_t ystride, double2* z, int64_t zstride, int ncol, const int* active,
                       int by_multiplicity);

// block GMRES: split-K Gram reduction, Cholesky + inverse of a p x p Gram
// matrix, block Hessenberg least-squares step and back substitution
// cond (device flag, optional): the launch does its work only when *cond != 0
void launch_gram_reduce(hipStream_t st, int64_t len, int nparts, const double2* part, double2* H,
                        const int* cond = nullptr);
void launch_bgram(hipStream_t st, const double2* V, int Q, const double2* W, int p, int64_t n, int nchunks,
                  double2* part, const int* cond = nullptr);
int bgram_parts(int64_t n, int nchunks);
void launch_bupdate(hipStream_t st, const double2* A, int K, const double2* M, int ldm, int p, int64_t n,
                    double alpha, double beta, const double2* C, double2* out, const int* cond = nullptr);
void launch_chol(hipStream_t st, int p, const double2* G, double2* R, double2* Rinv, const double2* Rprev,
                 double2* S, int* info);
void launch_set_e(hipStream_t st, int p, int ldE, const double2* S0, double2* E);
// h2_used (device flag, optional): H2 counts only when *h2_used != 0
void launch_bls_step(hipStream_t st, int j, int p, int m, const double2* H1, const double2* H2, const double2* S,
                     double2* Hc, double2* T, double2* Rls, double2* E, double* est, const int* h2_used = nullptr);
void launch_bls_solve(hipStream_t st, int jp, int p, int m, const double2* Rls, const double2* E, double2* Y);
void launch_reorth_check(hipStream_t st, int p, const double2* G0, const double2* G1, int* flag);
int max_block_p();

void launch_spmv(hipStream_t st, int group, int64_t n, const int64_t* rowptr, const int* cols, const double2* vals,
                 const double2* x, int64_t xstride, double2* y, int64_t ystride, const double2* b, int64_t bstride,
                 int ncol, const int* active);

// y = A x (or b - A x) for p <= interleaved_cols() columns through an
// interleaved copy xi [n][interleaved_cols()] of x (scratch, written here);
// the matrix is read once for all columns
void launch_spmm_interleaved(hipStream_t st, int64_t n, int p, const int64_t* rowptr, const int* cols,
                             const double2* vals, const double2* x, int64_t xstride, double2* xi, double2* y,
                             int64_t ystride, const double2* b, int64_t bstride);
int interleaved_cols();
// xi[j][c] = x[c][j] for the p <= interleaved_cols() columns (stride xstride),
// columns p.. zero
void launch_to_interleaved(hipStream_t st, int64_t n, int p, const double2* x, int64_t xstride, double2* xi);

int red_blocks(int64_t ndof);
void launch_dots(hipStream_t st, int64_t ndof, int nvec, const double2* V, int64_t vcol, const double2* w,
                 int64_t wcol, double2* part, int maxv, int ncol, const int* active);
void launch_reduce_dots(hipStream_t st, int64_t ndof, int nvec, const double2* part, double2* h, int maxv,
                        int accumulate, int ncol, const int* active);
void launch_update(hipStream_t st, int64_t ndof, int nvec, const double2* V, int64_t vcol, double2* w, int64_t wcol,
                   const double2* hpass, int maxv, int ncol, const int* active);
void launch_norm(hipStream_t st, int64_t ndof, const double2* w, int64_t wcol, double* part, double* out, int ncol,
                 const int* active);
void launch_scale_inv(hipStream_t st, int64_t ndof, const double2* x, int64_t xcol, double2* y, int64_t ycol,
                      const double* norm, int ncol, const int* active);
void launch_givens(hipStream_t st, int ncol, int j, int maxv, const double2* h, const double* hn, double2* H, int ldh,
                   double* cs, double2* sn, double2* g, double* est, const int* active);
void launch_backsolve(hipStream_t st, int ncol, const int* jd, int maxv, const double2* H, int ldh, const double2* g,
                      double2* y);
void launch_xupdate(hipStream_t st, int64_t ndof, const int* jd, const double2* Z, int64_t zcol, const double2* y,
                    int maxv, double2* x, int64_t xcol, int ncol);

// Krylov subspace recycling (GCRO-DR): Gbar columns, the recycled part of
// the least-squares solution, and the deflated restart of a cycle
constexpr int kRecycleMaxCycle = 64;   // largest recycled + Arnoldi vectors per cycle
constexpr int kRecycleLd = kRecycleMaxCycle + 1;
constexpr int kRecycleMaxK = 32;       // largest recycled dimension
constexpr int kRecycleMaxBlockP = 16;  // widest block of Block GCRO-DR
void launch_rc_save(hipStream_t st, int kk, int j, const double2* h, const double* hn, double2* G);
void launch_rc_by(hipStream_t st, int kk, const int* jd, const double2* G, const double2* y, double2* t);
void launch_rc_ritz(hipStream_t st, int kk, int jd, int knew, int extra, int ldw, const double2* G,
                    const double2* WVg, const double2* UU, double2* Mc, double2* Mu, double2* mu, int* info);
void launch_rc_save_block(hipStream_t st, int kk, int j, int p, const double2* B1, const double2* B2,
                          const double2* H1, const double2* H2, const double2* S, double2* G);
void launch_rc_by_block(hipStream_t st, int kk, int q, int p, const double2* G, const double2* Y, int ldy,
                        double2* T);

}  // namespace mxw
