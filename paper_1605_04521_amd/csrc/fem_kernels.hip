// Finite element kernels (FP64): element matrices, impedance face matrices,
// deterministic CSR assembly of A, dense local matrices A_s, right-hand sides.
//
// Weak form (Sec. 2, written for exp(-i w t)):
//   int curl E . curl v - k0^2 eps E . v - i beta int_Gamma E_t . v_t = int_Gamma g . v
// so A_T = K_T - k0^2 eps_T M_T per element and -i beta B_F per impedance face,
// with K_T = int curl phi_p . curl phi_q, M_T = int phi_p . phi_q and
// B_F = int_F (phi_p)_t . (phi_q)_t.  Integrals of barycentric monomials are
// exact: int_T lambda^a = 6|T| a!/(|a|+3)!, int_F mu^a = 2|F| a!/(|a|+2)!.
#include "device.h"
#include "kernels.h"

namespace mxw {

__constant__ double c_fact[16] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0, 5040.0, 40320.0,
                                  362880.0, 3628800.0, 39916800.0, 479001600.0,
                                  6227020800.0, 87178291200.0, 1307674368000.0};

__device__ __forceinline__ double tet_moment(const int8_t* a, const int8_t* b) {
  int s0 = a[0] + b[0], s1 = a[1] + b[1], s2 = a[2] + b[2], s3 = a[3] + b[3];
  return 6.0 * c_fact[s0] * c_fact[s1] * c_fact[s2] * c_fact[s3] / c_fact[s0 + s1 + s2 + s3 + 3];
}

__device__ __forceinline__ double face_moment(const int8_t* a, const int8_t* b) {
  int s0 = a[0] + b[0], s1 = a[1] + b[1], s2 = a[2] + b[2];
  return 2.0 * c_fact[s0] * c_fact[s1] * c_fact[s2] / c_fact[s0 + s1 + s2 + 2];
}

__device__ __forceinline__ int pair_index(int u, int v) {  // (u<v) -> 0..5
  return u * (7 - u) / 2 + v - u - 1;
}

// Barycentric gradients g[4][3] and volume of the tet with vertices X[4][3].
__device__ void tet_gradients(const double X[4][3], double g[4][3], double* vol) {
  double J[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) J[r][c] = X[c + 1][r] - X[0][r];   // columns X_i - X_0
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
               J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  double id = 1.0 / det;
  // rows of J^{-1} are grad lambda_1..3
  double inv[3][3];
  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  for (int c = 0; c < 3; ++c) {
    g[1][c] = inv[0][c];
    g[2][c] = inv[1][c];
    g[3][c] = inv[2][c];
    g[0][c] = -(inv[0][c] + inv[1][c] + inv[2][c]);
  }
  *vol = fabs(det) / 6.0;
}

// One block per element: A_T[p][q] = K_T - k0^2 eps_T M_T.
__global__ void __launch_bounds__(256) k_element(const double* __restrict__ xyz, const int* __restrict__ tets,
                                                 const double* __restrict__ eps, const Term* __restrict__ phi,
                                                 const Term* __restrict__ curl, int nloc, int ncurl,
                                                 double k0sq, double2* __restrict__ AT) {
  const int64_t t = blockIdx.x;
  __shared__ double G[4][4];
  __shared__ double C[6][6];
  __shared__ double X[6][3];
  __shared__ double vol_s;
  if (threadIdx.x == 0) {
    double P[4][3], g[4][3], vol;
    for (int q = 0; q < 4; ++q)
      for (int c = 0; c < 3; ++c) P[q][c] = xyz[3 * (int64_t)tets[4 * t + q] + c];
    tet_gradients(P, g, &vol);
    for (int u = 0; u < 4; ++u)
      for (int v = 0; v < 4; ++v) G[u][v] = g[u][0] * g[v][0] + g[u][1] * g[v][1] + g[u][2] * g[v][2];
    const int pu[6] = {0, 0, 0, 1, 1, 2}, pv[6] = {1, 2, 3, 2, 3, 3};
    for (int a = 0; a < 6; ++a) {
      const double* gu = g[pu[a]];
      const double* gv = g[pv[a]];
      X[a][0] = gu[1] * gv[2] - gu[2] * gv[1];
      X[a][1] = gu[2] * gv[0] - gu[0] * gv[2];
      X[a][2] = gu[0] * gv[1] - gu[1] * gv[0];
    }
    vol_s = vol;
  }
  __syncthreads();
  if (threadIdx.x < 36) {
    int a = threadIdx.x / 6, b = threadIdx.x % 6;
    C[a][b] = X[a][0] * X[b][0] + X[a][1] * X[b][1] + X[a][2] * X[b][2];
  }
  __syncthreads();
  const double vol = vol_s;
  const double er = eps[2 * t], ei = eps[2 * t + 1];
  for (int pq = threadIdx.x; pq < nloc * nloc; pq += blockDim.x) {
    const int p = pq / nloc, q = pq % nloc;
    double m = 0.0, k = 0.0;
#pragma unroll
    for (int a = 0; a < kMaxPhiTerms; ++a)
#pragma unroll
      for (int b = 0; b < kMaxPhiTerms; ++b) {
        const Term& s = phi[p * kMaxPhiTerms + a];
        const Term& u = phi[q * kMaxPhiTerms + b];
        m += s.coef * u.coef * tet_moment(s.alpha, u.alpha) * G[s.u][u.u];
      }
    for (int a = 0; a < ncurl; ++a) {
      const Term& s = curl[p * kMaxCurlTerms + a];
      if (s.coef == 0.0) continue;
      const int ia = pair_index(s.u, s.v);
      for (int b = 0; b < ncurl; ++b) {
        const Term& u = curl[q * kMaxCurlTerms + b];
        if (u.coef == 0.0) continue;
        k += s.coef * u.coef * tet_moment(s.alpha, u.alpha) * C[ia][pair_index(u.u, u.v)];
      }
    }
    m *= vol;
    k *= vol;
    AT[(t * nloc + p) * nloc + q] = make_double2(k - k0sq * er * m, -k0sq * ei * m);
  }
}

// Surface barycentric gradients of the triangle Y[3][3] and its area.
__device__ void face_gradients(const double Y[3][3], double g[3][3], double* area, double nrm[3]) {
  double e1[3], e2[3];
  for (int c = 0; c < 3; ++c) {
    e1[c] = Y[1][c] - Y[0][c];
    e2[c] = Y[2][c] - Y[0][c];
  }
  double a11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
  double a12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
  double a22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
  double det = a11 * a22 - a12 * a12;
  double i11 = a22 / det, i12 = -a12 / det, i22 = a11 / det;
  for (int c = 0; c < 3; ++c) {
    g[1][c] = i11 * e1[c] + i12 * e2[c];
    g[2][c] = i12 * e1[c] + i22 * e2[c];
    g[0][c] = -g[1][c] - g[2][c];
  }
  nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
  nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
  nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
  double nn = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
  *area = 0.5 * nn;
  for (int c = 0; c < 3; ++c) nrm[c] /= nn;
}

// One block per table face: B_F over the face-local generators.
__global__ void __launch_bounds__(256) k_face(const double* __restrict__ xyz, const int* __restrict__ fvert,
                                              const Term* __restrict__ fphi, int nfloc,
                                              double* __restrict__ BF) {
  const int64_t f = blockIdx.x;
  __shared__ double GF[3][3];
  __shared__ double area_s;
  if (threadIdx.x == 0) {
    double Y[3][3], g[3][3], area, nrm[3];
    for (int q = 0; q < 3; ++q)
      for (int c = 0; c < 3; ++c) Y[q][c] = xyz[3 * (int64_t)fvert[3 * f + q] + c];
    face_gradients(Y, g, &area, nrm);
    for (int u = 0; u < 3; ++u)
      for (int v = 0; v < 3; ++v) GF[u][v] = g[u][0] * g[v][0] + g[u][1] * g[v][1] + g[u][2] * g[v][2];
    area_s = area;
  }
  __syncthreads();
  for (int pq = threadIdx.x; pq < nfloc * nfloc; pq += blockDim.x) {
    const int p = pq / nfloc, q = pq % nfloc;
    double b = 0.0;
#pragma unroll
    for (int a = 0; a < kMaxPhiTerms; ++a)
#pragma unroll
      for (int c = 0; c < kMaxPhiTerms; ++c) {
        const Term& s = fphi[p * kMaxPhiTerms + a];
        const Term& u = fphi[q * kMaxPhiTerms + c];
        b += s.coef * u.coef * face_moment(s.alpha, u.alpha) * GF[s.u][u.u];
      }
    BF[(f * nfloc + p) * nfloc + q] = area_s * b;
  }
}

__device__ __forceinline__ int64_t find_col(const int* __restrict__ cols, int64_t lo, int64_t hi, int c) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (cols[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One thread per row: sums the row's element and face contributions in a
// fixed order (element ids ascending, then impedance faces) -- no atomics.
__global__ void k_assemble_rows(int64_t ndof, const int64_t* __restrict__ rowptr, const int* __restrict__ cols,
                                const int* __restrict__ dof_ent, const int64_t* __restrict__ ent_tet_ptr,
                                const int* __restrict__ ent_tets, const int64_t* __restrict__ ent_imp_ptr,
                                const int* __restrict__ ent_imps, const int* __restrict__ tet_dofs, int nloc,
                                const double2* __restrict__ AT, const int* __restrict__ imp_ft,
                                const double* __restrict__ imp_beta, const int* __restrict__ ft_dofs,
                                int nfloc, const double* __restrict__ BF, double2* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndof) return;
  const int64_t r0 = rowptr[i], r1 = rowptr[i + 1];
  for (int64_t c = r0; c < r1; ++c) vals[c] = make_double2(0.0, 0.0);
  const int en = dof_ent[i];
  for (int64_t q = ent_tet_ptr[en]; q < ent_tet_ptr[en + 1]; ++q) {
    const int64_t t = ent_tets[q];
    const int* td = tet_dofs + t * nloc;
    int p = 0;
    while (p < nloc && td[p] != (int)i) ++p;
    if (p == nloc) continue;
    const double2* a = AT + (t * nloc + p) * nloc;
    for (int qq = 0; qq < nloc; ++qq) {
      int c = td[qq];
      if (c < 0) continue;
      int64_t s = find_col(cols, r0, r1, c);
      if (s >= r1 || cols[s] != c) continue;
      double2 v = vals[s];
      v.x += a[qq].x;
      v.y += a[qq].y;
      vals[s] = v;
    }
  }
  for (int64_t q = ent_imp_ptr[en]; q < ent_imp_ptr[en + 1]; ++q) {
    const int k = ent_imps[q];
    const int64_t f = imp_ft[k];
    const double beta = imp_beta[k];
    const int* fd = ft_dofs + f * nfloc;
    int p = 0;
    while (p < nfloc && fd[p] != (int)i) ++p;
    if (p == nfloc) continue;
    const double* b = BF + (f * nfloc + p) * nfloc;
    for (int qq = 0; qq < nfloc; ++qq) {
      int c = fd[qq];
      if (c < 0) continue;
      int64_t s = find_col(cols, r0, r1, c);
      if (s >= r1 || cols[s] != c) continue;
      vals[s].y -= beta * b[qq];
    }
  }
}

// One block per subdomain: dense column-major A_s in the factor precision R,
// split planes (real part, then imaginary part), leading dimension ld.
// Elements are added one after another (block-wide barrier between them), then
// the original impedance faces and the interface faces (coefficient -i w~).
template <typename R>
__global__ void __launch_bounds__(256) k_assemble_local(
    R* __restrict__ F, const int64_t* __restrict__ foff, const int* __restrict__ nsz, const int* __restrict__ lds,
    const int64_t* __restrict__ tet_ptr, const int* __restrict__ tets, const int* __restrict__ lmap,
    const double2* __restrict__ AT, int nloc, const int64_t* __restrict__ face_ptr,
    const int* __restrict__ face_ft, const double* __restrict__ face_coef, const int* __restrict__ face_lmap,
    const double* __restrict__ BF, int nfloc, int with_ifaces, const int* __restrict__ list) {
  const int s = list ? list[blockIdx.x] : blockIdx.x;
  const int n = nsz[s], ld = lds[s];
  R* re = F + foff[s];
  R* im = re + (int64_t)ld * n;
  const int64_t tot = 2 * (int64_t)ld * n;
  for (int64_t q = threadIdx.x; q < tot; q += blockDim.x) re[q] = R(0);
  __syncthreads();
  const int nn = nloc * nloc;
  for (int64_t e = tet_ptr[s]; e < tet_ptr[s + 1]; ++e) {
    const int64_t t = tets[e];
    const int* lm = lmap + e * nloc;
    for (int pq = threadIdx.x; pq < nn; pq += blockDim.x) {
      const int p = pq / nloc, q = pq % nloc;
      const int i = lm[p], j = lm[q];
      if (i < 0 || j < 0) continue;
      const double2 a = AT[t * nn + pq];
      const int64_t o = (int64_t)j * ld + i;
      re[o] = (R)((double)re[o] + a.x);
      im[o] = (R)((double)im[o] + a.y);
    }
    __syncthreads();
  }
  const int nf2 = nfloc * nfloc;
  for (int64_t e = face_ptr[s]; e < face_ptr[s + 1]; ++e) {
    const double coef = face_coef[e];
    const int64_t f = face_ft[e];
    const int* lm = face_lmap + e * nfloc;
    // faces of the original boundary come first and are always added; the
    // interface faces are recognised by the caller-provided flag array
    for (int pq = threadIdx.x; pq < nf2; pq += blockDim.x) {
      const int p = pq / nfloc, q = pq % nfloc;
      const int i = lm[p], j = lm[q];
      if (i < 0 || j < 0) continue;
      const int64_t o = (int64_t)j * ld + i;
      im[o] = (R)((double)im[o] - coef * BF[f * nf2 + pq]);
    }
    __syncthreads();
  }
  (void)with_ifaces;
}

// Dipole right-hand side: b[c][dof_p] += pol . phi_p(lambda) in one element.
__global__ void k_rhs_dipole(const double* __restrict__ xyz, const int* __restrict__ tets,
                             const int* __restrict__ tet_dofs, const Term* __restrict__ phi, int nloc,
                             int64_t t, double l0, double l1, double l2, double l3, double pr0, double pr1,
                             double pr2, double pi0, double pi1, double pi2, double2* __restrict__ b) {
  const int p = threadIdx.x;
  if (p >= nloc) return;
  double P[4][3], g[4][3], vol;
  for (int q = 0; q < 4; ++q)
    for (int c = 0; c < 3; ++c) P[q][c] = xyz[3 * (int64_t)tets[4 * t + q] + c];
  tet_gradients(P, g, &vol);
  const double lam[4] = {l0, l1, l2, l3};
  double val[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < kMaxPhiTerms; ++a) {
    const Term& s = phi[p * kMaxPhiTerms + a];
    double mono = s.coef;
    for (int m = 0; m < 4; ++m)
      for (int e = 0; e < s.alpha[m]; ++e) mono *= lam[m];
    for (int c = 0; c < 3; ++c) val[c] += mono * g[s.u][c];
  }
  const int d = tet_dofs[t * nloc + p];
  if (d < 0) return;
  double2 v = b[d];
  v.x += pr0 * val[0] + pr1 * val[1] + pr2 * val[2];
  v.y += pi0 * val[0] + pi1 * val[1] + pi2 * val[2];
  b[d] = v;
}

__device__ __forceinline__ double2 csqrt_principal(double a, double b) {
  double r = hypot(a, b);
  double re = sqrt(0.5 * (r + a));
  double im = sqrt(fmax(0.0, 0.5 * (r - a)));
  return make_double2(re, b < 0 ? -im : im);
}

// Plane-wave boundary data on impedance faces, one thread per face:
// g = (curl E) x n - i beta n x (E x n), E = p exp(i kappa d.x),
// kappa = k0 sqrt(eps) of the adjacent element, curl E = i kappa d x E;
// out[f][p] = int_F g . phi_p with the collapsed Gauss-Legendre rule
// (mu1 = xi(1-eta), mu2 = xi eta, weight 2|F| w w xi).
__global__ void k_rhs_planewave(int nimp, const double* __restrict__ xyz, const int* __restrict__ fvert,
                                const int* __restrict__ imp_ft, const int* __restrict__ imp_opp,
                                const double* __restrict__ imp_beta, const double* __restrict__ imp_eps,
                                const Term* __restrict__ fphi, int nfloc, double k0, int nq,
                                const double* __restrict__ gx, const double* __restrict__ gw, double pr0,
                                double pr1, double pr2, double pi0, double pi1, double pi2, double d0, double d1,
                                double d2, double2* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nimp) return;
  const int64_t f = imp_ft[k];
  double Y[3][3], g[3][3], area, nrm[3];
  for (int q = 0; q < 3; ++q)
    for (int c = 0; c < 3; ++c) Y[q][c] = xyz[3 * (int64_t)fvert[3 * f + q] + c];
  face_gradients(Y, g, &area, nrm);
  {  // orient the normal away from the element's fourth vertex
    const double* O = xyz + 3 * (int64_t)imp_opp[k];
    double dd = (O[0] - Y[0][0]) * nrm[0] + (O[1] - Y[0][1]) * nrm[1] + (O[2] - Y[0][2]) * nrm[2];
    if (dd > 0)
      for (int c = 0; c < 3; ++c) nrm[c] = -nrm[c];
  }
  const double beta = imp_beta[k];
  const double2 kap0 = csqrt_principal(imp_eps[2 * k], imp_eps[2 * k + 1]);
  const double kr = k0 * kap0.x, ki = k0 * kap0.y;
  double accr[kMaxFaceLoc], acci[kMaxFaceLoc];
  for (int p = 0; p < kMaxFaceLoc; ++p) accr[p] = acci[p] = 0.0;
  const double d[3] = {d0, d1, d2};
  for (int a = 0; a < nq; ++a)
    for (int b = 0; b < nq; ++b) {
      const double xi = gx[a], eta = gx[b];
      const double mu[3] = {1.0 - xi, xi * (1.0 - eta), xi * eta};
      const double w = 2.0 * area * gw[a] * gw[b] * xi;
      double x[3];
      for (int c = 0; c < 3; ++c) x[c] = mu[0] * Y[0][c] + mu[1] * Y[1][c] + mu[2] * Y[2][c];
      const double s = d[0] * x[0] + d[1] * x[1] + d[2] * x[2];
      // exp(i kappa s) = exp(-ki s) (cos(kr s) + i sin(kr s))
      const double amp = exp(-ki * s);
      const double er = amp * cos(kr * s), ei = amp * sin(kr * s);
      double Er[3], Ei[3];
      const double pr[3] = {pr0, pr1, pr2}, pim[3] = {pi0, pi1, pi2};
      for (int c = 0; c < 3; ++c) {
        Er[c] = pr[c] * er - pim[c] * ei;
        Ei[c] = pr[c] * ei + pim[c] * er;
      }
      // curl E = i kappa (d x E)
      double dxr[3] = {d[1] * Er[2] - d[2] * Er[1], d[2] * Er[0] - d[0] * Er[2], d[0] * Er[1] - d[1] * Er[0]};
      double dxi[3] = {d[1] * Ei[2] - d[2] * Ei[1], d[2] * Ei[0] - d[0] * Ei[2], d[0] * Ei[1] - d[1] * Ei[0]};
      double cr[3], ci[3];
      for (int c = 0; c < 3; ++c) {   // (i kappa) * (dxr + i dxi), i kappa = -ki + i kr
        cr[c] = -ki * dxr[c] - kr * dxi[c];
        ci[c] = -ki * dxi[c] + kr * dxr[c];
      }
      // (curl E) x n
      double gr[3] = {cr[1] * nrm[2] - cr[2] * nrm[1], cr[2] * nrm[0] - cr[0] * nrm[2], cr[0] * nrm[1] - cr[1] * nrm[0]};
      double gi[3] = {ci[1] * nrm[2] - ci[2] * nrm[1], ci[2] * nrm[0] - ci[0] * nrm[2], ci[0] * nrm[1] - ci[1] * nrm[0]};
      // - i beta E_t, E_t = E - (E.n) n
      const double enr = Er[0] * nrm[0] + Er[1] * nrm[1] + Er[2] * nrm[2];
      const double eni = Ei[0] * nrm[0] + Ei[1] * nrm[1] + Ei[2] * nrm[2];
      for (int c = 0; c < 3; ++c) {
        const double tr = Er[c] - enr * nrm[c], ti = Ei[c] - eni * nrm[c];
        gr[c] += beta * ti;
        gi[c] -= beta * tr;
      }
      for (int p = 0; p < nfloc; ++p) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int t = 0; t < kMaxPhiTerms; ++t) {
          const Term& tm = fphi[p * kMaxPhiTerms + t];
          double mono = tm.coef;
          for (int m = 0; m < 3; ++m)
            for (int e = 0; e < tm.alpha[m]; ++e) mono *= mu[m];
          for (int c = 0; c < 3; ++c) v[c] += mono * g[tm.u][c];
        }
        accr[p] += w * (gr[0] * v[0] + gr[1] * v[1] + gr[2] * v[2]);
        acci[p] += w * (gi[0] * v[0] + gi[1] * v[1] + gi[2] * v[2]);
      }
    }
  for (int p = 0; p < nfloc; ++p) out[(int64_t)k * nfloc + p] = make_double2(accr[p], acci[p]);
}

// b[i] += sum over the impedance faces of i's entity of their contribution.
// Rectangular port with the TE10 mode (eq. (3), eq. (5)).  A face belongs to
// the port when its centroid lies in the rectangle c + s u + t v, |s| <= a/2,
// |t| <= b/2 (within 1e-9 (a + b), also off the plane).  The mode on the
// port is E0 = sin(pi (s + a/2) / a) v.
//   mode 0: face integrals of g . phi_p, g = -i (beta10 + beta) E0 (the
//           excitation; beta10 = sqrt(max(beta^2 - (pi/a)^2, 0)))
//   mode 1: face integrals of E0 . phi_p (the S-matrix weights) and, per
//           face, the integral of |E0|^2 in fnorm
// Faces outside the port write zeros.
__global__ void k_rhs_port(int nimp, const double* __restrict__ xyz, const int* __restrict__ fvert,
                           const int* __restrict__ imp_ft, const double* __restrict__ imp_beta,
                           const Term* __restrict__ fphi, int nfloc, int nq, const double* __restrict__ gx,
                           const double* __restrict__ gw, double c0, double c1, double c2, double u0, double u1,
                           double u2, double v0, double v1, double v2, double aw, double bh, int mode,
                           double2* __restrict__ out, double* __restrict__ fnorm) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nimp) return;
  const int64_t f = imp_ft[k];
  double Y[3][3], g[3][3], area, nrm[3];
  for (int q = 0; q < 3; ++q)
    for (int c = 0; c < 3; ++c) Y[q][c] = xyz[3 * (int64_t)fvert[3 * f + q] + c];
  face_gradients(Y, g, &area, nrm);
  const double cen[3] = {c0, c1, c2}, u[3] = {u0, u1, u2}, v[3] = {v0, v1, v2};
  const double pn[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  double ds = 0.0, dt = 0.0, dn = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double x = (Y[0][c] + Y[1][c] + Y[2][c]) / 3.0 - cen[c];
    ds += x * u[c];
    dt += x * v[c];
    dn += x * pn[c];
  }
  const double tol = 1e-9 * (aw + bh);
  const bool in = fabs(dn) <= tol && fabs(ds) <= 0.5 * aw + tol && fabs(dt) <= 0.5 * bh + tol;
  if (!in) {
    for (int p = 0; p < nfloc; ++p) out[(int64_t)k * nfloc + p] = make_double2(0.0, 0.0);
    if (fnorm) fnorm[k] = 0.0;
    return;
  }
  const double beta = imp_beta[k];
  const double kc = M_PI / aw;
  const double b10 = sqrt(fmax(beta * beta - kc * kc, 0.0));
  // the factor multiplying E0: -i (beta10 + beta) or 1
  const double fr = mode == 0 ? 0.0 : 1.0, fi = mode == 0 ? -(b10 + beta) : 0.0;
  double accr[kMaxFaceLoc], acci[kMaxFaceLoc];
  for (int p = 0; p < kMaxFaceLoc; ++p) accr[p] = acci[p] = 0.0;
  double fn = 0.0;
  for (int a = 0; a < nq; ++a)
    for (int b = 0; b < nq; ++b) {
      const double xi = gx[a], eta = gx[b];
      const double mu[3] = {1.0 - xi, xi * (1.0 - eta), xi * eta};
      const double w = 2.0 * area * gw[a] * gw[b] * xi;
      double s = 0.0;
      for (int c = 0; c < 3; ++c) s += (mu[0] * Y[0][c] + mu[1] * Y[1][c] + mu[2] * Y[2][c] - cen[c]) * u[c];
      const double prof = sin(kc * (s + 0.5 * aw));
      fn += w * prof * prof;
      for (int p = 0; p < nfloc; ++p) {
        double ph[3] = {0.0, 0.0, 0.0};
        for (int t = 0; t < kMaxPhiTerms; ++t) {
          const Term& tm = fphi[p * kMaxPhiTerms + t];
          double mono = tm.coef;
          for (int m = 0; m < 3; ++m)
            for (int e = 0; e < tm.alpha[m]; ++e) mono *= mu[m];
          for (int c = 0; c < 3; ++c) ph[c] += mono * g[tm.u][c];
        }
        const double pv = w * prof * (ph[0] * v[0] + ph[1] * v[1] + ph[2] * v[2]);
        accr[p] += fr * pv;
        acci[p] += fi * pv;
      }
    }
  for (int p = 0; p < nfloc; ++p) out[(int64_t)k * nfloc + p] = make_double2(accr[p], acci[p]);
  if (fnorm) fnorm[k] = fn;
}

// out[0] = sum of x[0..n) (one block, fixed order)
__global__ void k_sum_fixed(int n, const double* __restrict__ x, double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += x[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// S[(i0 + i) nsol + j] = num[i nsol + j] / den[i]
__global__ void k_smatrix_finish(int nsol, int np, const double2* __restrict__ num, const double* __restrict__ den,
                                 double2* __restrict__ S) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nsol * np) return;
  const int i = e / nsol;
  const double d = den[i];
  S[e] = make_double2(num[e].x / d, num[e].y / d);
}

__global__ void k_gather_face_rhs(int64_t ndof, const int* __restrict__ dof_ent, const int64_t* __restrict__ ent_imp_ptr,
                                  const int* __restrict__ ent_imps, const int* __restrict__ imp_ft,
                                  const int* __restrict__ ft_dofs, int nfloc, const double2* __restrict__ fr,
                                  double2* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndof) return;
  const int en = dof_ent[i];
  double2 acc = b[i];
  for (int64_t q = ent_imp_ptr[en]; q < ent_imp_ptr[en + 1]; ++q) {
    const int k = ent_imps[q];
    const int* fd = ft_dofs + (int64_t)imp_ft[k] * nfloc;
    for (int p = 0; p < nfloc; ++p)
      if (fd[p] == (int)i) {
        acc.x += fr[(int64_t)k * nfloc + p].x;
        acc.y += fr[(int64_t)k * nfloc + p].y;
      }
  }
  b[i] = acc;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

void launch_element(hipStream_t st, int64_t nt, const double* xyz, const int* tets, const double* eps,
                    const Term* phi, const Term* curl, int nloc, int ncurl, double k0sq, double2* AT) {
  if (nt > 0) hipLaunchKernelGGL(k_element, dim3((unsigned)nt), dim3(256), 0, st, xyz, tets, eps, phi, curl, nloc, ncurl, k0sq, AT);
}

void launch_face(hipStream_t st, int64_t nft, const double* xyz, const int* fvert, const Term* fphi, int nfloc,
                 double* BF) {
  if (nft > 0) hipLaunchKernelGGL(k_face, dim3((unsigned)nft), dim3(256), 0, st, xyz, fvert, fphi, nfloc, BF);
}

void launch_assemble_rows(hipStream_t st, const AssembleArgs& a) {
  if (a.ndof == 0) return;
  const unsigned nb = (unsigned)((a.ndof + 127) / 128);
  hipLaunchKernelGGL(k_assemble_rows, dim3(nb), dim3(128), 0, st, a.ndof, a.rowptr, a.cols, a.dof_ent, a.ent_tet_ptr,
                     a.ent_tets, a.ent_imp_ptr, a.ent_imps, a.tet_dofs, a.nloc, a.AT, a.imp_ft, a.imp_beta,
                     a.ft_dofs, a.nfloc, a.BF, a.vals);
}

// Dirichlet transmission (RAS, Sec. 4): A_s = R_s A R_s^T, the principal
// submatrix of the assembled global matrix on the subdomain's unknowns.  One
// workgroup per subdomain: the dense matrix is cleared, then each local row
// scans its global CSR row and places the entries whose column belongs to the
// subdomain (binary search in the sorted unknown list).
template <typename R>
__global__ void __launch_bounds__(256) k_local_from_csr(R* __restrict__ F, const int64_t* __restrict__ foff,
                                                        const int* __restrict__ nsz, const int* __restrict__ lds,
                                                        const int64_t* __restrict__ poff,
                                                        const int* __restrict__ sub_dofs,
                                                        const int64_t* __restrict__ rowptr,
                                                        const int* __restrict__ cols,
                                                        const double2* __restrict__ vals) {
  const int s = blockIdx.x;
  const int n = nsz[s], ld = lds[s];
  R* re = F + foff[s];
  R* im = re + (int64_t)ld * n;
  const int64_t tot = 2 * (int64_t)ld * n;
  for (int64_t q = threadIdx.x; q < tot; q += blockDim.x) re[q] = R(0);
  __syncthreads();
  const int* D = sub_dofs + poff[s];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int g = D[i];
    for (int64_t e = rowptr[g]; e < rowptr[g + 1]; ++e) {
      const int c = cols[e];
      int lo = 0, hi = n;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (D[mid] < c)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo < n && D[lo] == c) {
        const double2 a = vals[e];
        re[(int64_t)lo * ld + i] = (R)a.x;
        im[(int64_t)lo * ld + i] = (R)a.y;
      }
    }
  }
}

template <typename R>
void launch_local_from_csr(hipStream_t st, int n_sub, R* F, const int64_t* foff, const int* nsz, const int* lds,
                           const int64_t* poff, const int* sub_dofs, const int64_t* rowptr, const int* cols,
                           const double2* vals) {
  if (n_sub == 0) return;
  hipLaunchKernelGGL(k_local_from_csr<R>, dim3(n_sub), dim3(256), 0, st, F, foff, nsz, lds, poff, sub_dofs, rowptr,
                     cols, vals);
}
template void launch_local_from_csr<double>(hipStream_t, int, double*, const int64_t*, const int*, const int*,
                                            const int64_t*, const int*, const int64_t*, const int*, const double2*);
template void launch_local_from_csr<float>(hipStream_t, int, float*, const int64_t*, const int*, const int*,
                                           const int64_t*, const int*, const int64_t*, const int*, const double2*);

template <typename R>
void launch_assemble_local(hipStream_t st, const LocalAssembleArgs& a, R* F) {
  if (a.n_sub == 0) return;
  hipLaunchKernelGGL(k_assemble_local<R>, dim3(a.n_sub), dim3(256), 0, st, F, a.foff, a.nsz, a.lds, a.tet_ptr,
                     a.tets, a.lmap, a.AT, a.nloc, a.face_ptr, a.face_ft, a.face_coef, a.face_lmap, a.BF,
                     a.nfloc, 1, a.list);
}
template void launch_assemble_local<double>(hipStream_t, const LocalAssembleArgs&, double*);
template void launch_assemble_local<float>(hipStream_t, const LocalAssembleArgs&, float*);

void launch_rhs_dipole(hipStream_t st, const double* xyz, const int* tets, const int* tet_dofs, const Term* phi,
                       int nloc, int64_t t, const double lam[4], const double pr[3], const double pi[3],
                       double2* b) {
  hipLaunchKernelGGL(k_rhs_dipole, dim3(1), dim3(64), 0, st, xyz, tets, tet_dofs, phi, nloc, t, lam[0], lam[1],
                     lam[2], lam[3], pr[0], pr[1], pr[2], pi[0], pi[1], pi[2], b);
}

void launch_rhs_port(hipStream_t st, const PlaneWaveArgs& a, const double c[3], const double u[3], const double v[3],
                     double aw, double bh, int mode, double2* work, double* fnorm, double* den, double2* b) {
  if (a.nimp == 0) {   // b (accumulated into) stays as it is
    if (den) hipMemsetAsync(den, 0, sizeof(double), st);
    return;
  }
  hipLaunchKernelGGL(k_rhs_port, dim3((a.nimp + 63) / 64), dim3(64), 0, st, a.nimp, a.xyz, a.fvert, a.imp_ft,
                     a.imp_beta, a.fphi, a.nfloc, a.nq, a.gx, a.gw, c[0], c[1], c[2], u[0], u[1], u[2], v[0], v[1],
                     v[2], aw, bh, mode, work, fnorm);
  hipLaunchKernelGGL(k_gather_face_rhs, dim3((unsigned)((a.ndof + 255) / 256)), dim3(256), 0, st, a.ndof, a.dof_ent,
                     a.ent_imp_ptr, a.ent_imps, a.imp_ft, a.ft_dofs, a.nfloc, work, b);
  if (den && fnorm) hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, a.nimp, fnorm, den);
}

void launch_smatrix_finish(hipStream_t st, int nsol, int np, const double2* num, const double* den, double2* S) {
  const int tot = nsol * np;
  hipLaunchKernelGGL(k_smatrix_finish, dim3((tot + 255) / 256), dim3(256), 0, st, nsol, np, num, den, S);
}

void launch_rhs_planewave(hipStream_t st, const PlaneWaveArgs& a, const double pr[3], const double pi[3],
                          const double d[3], double2* work, double2* b) {
  if (a.nimp == 0) return;
  hipLaunchKernelGGL(k_rhs_planewave, dim3((a.nimp + 63) / 64), dim3(64), 0, st, a.nimp, a.xyz, a.fvert, a.imp_ft,
                     a.imp_opp, a.imp_beta, a.imp_eps, a.fphi, a.nfloc, a.k0, a.nq, a.gx, a.gw, pr[0], pr[1], pr[2],
                     pi[0], pi[1], pi[2], d[0], d[1], d[2], work);
  hipLaunchKernelGGL(k_gather_face_rhs, dim3((unsigned)((a.ndof + 255) / 256)), dim3(256), 0, st, a.ndof, a.dof_ent,
                     a.ent_imp_ptr, a.ent_imps, a.imp_ft, a.ft_dofs, a.nfloc, work, b);
}

}  // namespace mxw
