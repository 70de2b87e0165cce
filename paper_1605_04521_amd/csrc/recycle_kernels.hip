// Krylov subspace recycling (GCRO-DR, the method Sec. 6 proposes for the
// slowly varying systems of the imaging loop): the small dense kernels of a
// cycle with recycled vectors and of the deflated restart.
//
// A cycle with kk recycled vectors C (A M^{-1} U = C, C^H C = I) and jd
// Arnoldi steps of (I - C C^H) A M^{-1} has  A M^{-1} [U D, V] = [C, V+] Gbar,
//   Gbar = [[D, B], [0, Hbar]]   ((kk + jd + 1) x (kk + jd)),
// D = diag(1 / |u_c|).  The new recycled space is spanned by the harmonic
// Ritz vectors of the kk + jd dimensional search space of largest 1 / theta,
// theta the eigenvalues of the pencil  Gbar^H Gbar z = theta Gbar^H WV z,
// WV = [C, V+]^H [U D, V].  With Gbar = Q R (Householder) the pencil becomes
// the ordinary problem  S z = (1 / theta) z,  S = R^{-1} Q^H WV; the kernel
// reduces S to complex Schur form, moves the selected eigenvalues to the
// front and takes P = the leading Schur vectors (the same span as their
// eigenvectors).  Then Gbar P = Qk Rk and the new space is
//   C <- [C, V+] Qk,   U <- [U D, V] P Rk^{-1}   (and Ubar likewise).
#include <hip/hip_runtime.h>

#include "device.h"
#include "kernels.h"

namespace mxw {

namespace {

constexpr int kRcMax = kRecycleMaxCycle;   // largest kk + jd
constexpr int kRcLd = kRecycleLd;          // leading dimension of the cycle matrices
constexpr int kRcK = kRecycleMaxK;         // largest recycled dimension

__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ double cabs_(double2 a) { return hypot(a.x, a.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 csqrt_(double2 z) {
  const double r = cabs_(z);
  double re = sqrt(0.5 * (r + z.x));
  double im = sqrt(0.5 * fmax(r - z.x, 0.0));
  if (z.y < 0) im = -im;
  return make_double2(re, im);
}

// Sum over the 256 threads of a block (4 waves); every thread gets the sum.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Complex Givens rotation (c real, s complex) with  c a + s b = r,
// -conj(s) a + c b = 0.
__device__ void givens_cs(double2 a, double2 b, double& c, double2& s) {
  const double na = cabs_(a), nb = cabs_(b);
  if (nb == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
  } else if (na == 0.0) {
    c = 0.0;
    s = cscale(cconj(b), 1.0 / nb);
  } else {
    const double nu = hypot(na, nb);
    c = na / nu;
    s = cscale(cmul(cscale(a, 1.0 / na), cconj(b)), 1.0 / nu);
  }
}

// Rotation of rows r, r+1 of the column-major matrix M (ld kRcLd), columns
// [c0, c1):  [x; y] <- [c s; -conj(s) c] [x; y].
__device__ void rot_rows(double2* M, int r, int c0, int c1, double c, double2 s) {
  for (int q = c0 + (int)threadIdx.x; q < c1; q += blockDim.x) {
    const double2 x = M[q * kRcLd + r], y = M[q * kRcLd + r + 1];
    M[q * kRcLd + r] = cadd(cscale(x, c), cmul(s, y));
    M[q * kRcLd + r + 1] = csub(cscale(y, c), cmul(cconj(s), x));
  }
}

// The matching similarity on columns r, r+1, rows [r0, r1):
// [x y] <- [x y] [c -s; conj(s) c]  (the conjugate transpose of the row rotation).
__device__ void rot_cols(double2* M, int r, int r0, int r1, double c, double2 s) {
  for (int i = r0 + (int)threadIdx.x; i < r1; i += blockDim.x) {
    const double2 x = M[r * kRcLd + i], y = M[(r + 1) * kRcLd + i];
    M[r * kRcLd + i] = cadd(cscale(x, c), cmul(cconj(s), y));
    M[(r + 1) * kRcLd + i] = csub(cscale(y, c), cmul(s, x));
  }
}

}  // namespace

// Column kk + j of Gbar from the Gram-Schmidt coefficients of step j:
// rows < kk + j + 1 are h (against C, then V_0..V_j), row kk + j + 1 is the
// norm of the remainder, the rest zero.
__global__ void k_rc_save(int kk, int j, const double2* __restrict__ h, const double* __restrict__ hn,
                          double2* __restrict__ G) {
  const int i = threadIdx.x;
  if (i >= kRcLd) return;
  const int top = kk + j + 1;
  double2 v = make_double2(0.0, 0.0);
  if (i < top) v = h[i];
  else if (i == top) v = make_double2(hn[0], 0.0);
  G[(int64_t)(kk + j) * kRcLd + i] = v;
}

// t = -B y: the recycled part of the least-squares solution (B = rows < kk
// of columns kk .. kk + jd - 1 of Gbar).
__global__ void k_rc_by(int kk, const int* __restrict__ jd, const double2* __restrict__ G, const double2* __restrict__ y,
                        double2* __restrict__ t) {
  const int i = threadIdx.x;
  if (i >= kk) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int c = 0; c < jd[0]; ++c) acc = cadd(acc, cmul(G[(int64_t)(kk + c) * kRcLd + i], y[c]));
  t[i] = make_double2(-acc.x, -acc.y);
}

// The deflated restart of one cycle (one workgroup of 256 threads).
//   G:   Gbar columns kk .. s-1 (ld kRcLd), columns < kk implied by D
//   WVg: [C, V_0..V_jd]^H U  ((s + extra) x kk, ld ldw)  (kk > 0)
//   UU:  U^H U  (kk x kk)                                   (kk > 0)
//   extra: rows of Gbar below s -- 1 for one right-hand side (0 after a
//   breakdown, where V_jd is not a basis vector), p for a block of p
// Outputs (ld kRcLd): Mc ((s + 1) x knew) with C_new = [C, V] Mc, and
// Mu (s x knew) with U_new = [U, V] Mu (D folded into its first kk rows);
// mu: the s values 1/theta, selected ones first; info[0] = 1 when the Schur
// iteration did not converge or a pivot vanished.
__global__ void __launch_bounds__(256) k_rc_ritz(int kk, int jd, int knew, int extra, int ldw,
                                                 const double2* __restrict__ G, const double2* __restrict__ WVg,
                                                 const double2* __restrict__ UU, double2* __restrict__ Mc,
                                                 double2* __restrict__ Mu, double2* __restrict__ mu,
                                                 int* __restrict__ info) {
  __shared__ double2 A1[kRcMax * kRcLd];   // Gbar -> R -> Schur vectors
  __shared__ double2 A2[kRcMax * kRcLd];   // WV -> S -> Schur form -> Gbar P -> Qk
  __shared__ double2 Rk[kRcK * kRcK];
  __shared__ double2 vh[kRcLd];
  __shared__ double dsc[kRcK];
  __shared__ double red[4];
  __shared__ int sel[1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int s = kk + jd;
  const int rows = s + extra;
  const double2 zero = make_double2(0.0, 0.0);
  if (tid == 0) bad = 0;
  for (int c = tid; c < kk; c += blockDim.x) dsc[c] = 1.0 / sqrt(fmax(UU[c * kk + c].x, 1e-300));
  __syncthreads();

  // Gbar and WV
  for (int e = tid; e < kRcMax * kRcLd; e += blockDim.x) {
    const int c = e / kRcLd, i = e % kRcLd;
    double2 g = zero, w = zero;
    if (c < s && i < rows) {
      if (c < kk) {
        g = (i == c) ? make_double2(dsc[c], 0.0) : zero;
        w = cscale(WVg[(int64_t)c * ldw + i], dsc[c]);
      } else {
        g = G[(int64_t)c * kRcLd + i];
        w = (i == c) ? make_double2(1.0, 0.0) : zero;
      }
    }
    A1[e] = g;
    A2[e] = w;
  }
  __syncthreads();

  // Householder QR of Gbar (rows x s), the reflectors applied to WV too:
  // afterwards A1 holds R (s x s) and rows < s of A2 hold Q^H WV
  for (int c = 0; c < s; ++c) {
    const int len = rows - c;
    double part = 0.0;
    for (int i = tid; i < len; i += blockDim.x) part += cabs2(A1[c * kRcLd + c + i]);
    const double nrm = sqrt(block_sum(part, red));
    for (int i = tid; i < len; i += blockDim.x) vh[i] = A1[c * kRcLd + c + i];
    __syncthreads();
    if (nrm == 0.0) continue;   // zero column: R_cc = 0 (flagged below)
    // v = x - alpha e1, alpha = -phase(x0) |x|; H = I - 2 v v^H / (v^H v)
    const double2 x0 = vh[0];
    const double a0 = cabs_(x0);
    const double2 ph = a0 > 0.0 ? cscale(x0, 1.0 / a0) : make_double2(1.0, 0.0);
    const double2 alpha = cscale(ph, -nrm);
    const double vnorm2 = 2.0 * nrm * (nrm + a0);   // |x - alpha e1|^2
    __syncthreads();
    if (tid == 0) vh[0] = csub(x0, alpha);
    __syncthreads();
    const double tau = 2.0 / vnorm2;
    // columns c+1.. of A1 and all s columns of A2
    for (int q = tid; q < 2 * s; q += blockDim.x) {
      double2* col = q < s ? A1 + q * kRcLd : A2 + (q - s) * kRcLd;
      if (q < s && q <= c) continue;
      double2 d = zero;
      for (int i = 0; i < len; ++i) d = cadd(d, conj_mul(vh[i], col[c + i]));
      d = cscale(d, tau);
      for (int i = 0; i < len; ++i) col[c + i] = csub(col[c + i], cmul(vh[i], d));
    }
    __syncthreads();
    if (tid == 0) A1[c * kRcLd + c] = alpha;
    for (int i = 1 + tid; i < len; i += blockDim.x) A1[c * kRcLd + c + i] = zero;
    __syncthreads();
  }
  for (int c = tid; c < s; c += blockDim.x)
    if (cabs_(A1[c * kRcLd + c]) == 0.0) bad = 1;
  __syncthreads();
  if (bad) {
    if (tid == 0) info[0] = 1;
    return;
  }

  // S = R^{-1} (Q^H WV), one column per thread, in place in A2
  for (int q = tid; q < s; q += blockDim.x) {
    double2* col = A2 + q * kRcLd;
    for (int i = s - 1; i >= 0; --i) {
      double2 t = col[i];
      for (int l = i + 1; l < s; ++l) t = csub(t, cmul(A1[l * kRcLd + i], col[l]));
      col[i] = cdiv(t, A1[i * kRcLd + i]);
    }
  }
  __syncthreads();
  // A1 <- identity (accumulated unitary)
  for (int e = tid; e < kRcMax * kRcLd; e += blockDim.x) {
    const int c = e / kRcLd, i = e % kRcLd;
    A1[e] = (i == c && c < s) ? make_double2(1.0, 0.0) : zero;
  }
  __syncthreads();

  // Hessenberg reduction of S by Householder reflectors, accumulated in A1
  for (int c = 0; c + 2 < s; ++c) {
    const int len = s - c - 1;
    double part = 0.0;
    for (int i = tid; i < len; i += blockDim.x) part += cabs2(A2[c * kRcLd + c + 1 + i]);
    const double nrm = sqrt(block_sum(part, red));
    for (int i = tid; i < len; i += blockDim.x) vh[i] = A2[c * kRcLd + c + 1 + i];
    __syncthreads();
    if (nrm == 0.0) continue;
    const double2 x0 = vh[0];
    const double a0 = cabs_(x0);
    const double2 ph = a0 > 0.0 ? cscale(x0, 1.0 / a0) : make_double2(1.0, 0.0);
    const double2 alpha = cscale(ph, -nrm);
    const double tau = 2.0 / (2.0 * nrm * (nrm + a0));
    __syncthreads();
    if (tid == 0) vh[0] = csub(x0, alpha);
    __syncthreads();
    // left: S <- H S, columns c..s-1, rows c+1..s-1
    for (int q = c + tid; q < s; q += blockDim.x) {
      double2* col = A2 + q * kRcLd + c + 1;
      double2 d = zero;
      for (int i = 0; i < len; ++i) d = cadd(d, conj_mul(vh[i], col[i]));
      d = cscale(d, tau);
      for (int i = 0; i < len; ++i) col[i] = csub(col[i], cmul(vh[i], d));
    }
    __syncthreads();
    // right: S <- S H (all rows) and Qacc <- Qacc H, columns c+1..s-1
    for (int r = tid; r < 2 * s; r += blockDim.x) {
      double2* M = r < s ? A2 : A1;
      const int i = r < s ? r : r - s;
      double2 d = zero;
      for (int l = 0; l < len; ++l) d = cadd(d, cmul(M[(c + 1 + l) * kRcLd + i], vh[l]));
      d = cscale(d, tau);
      for (int l = 0; l < len; ++l)
        M[(c + 1 + l) * kRcLd + i] = csub(M[(c + 1 + l) * kRcLd + i], cmul(d, cconj(vh[l])));
    }
    __syncthreads();
    for (int i = tid; i < len - 1; i += blockDim.x) A2[c * kRcLd + c + 2 + i] = zero;
    __syncthreads();
  }

  // Complex Schur form by single-shift QR sweeps (Wilkinson shift,
  // exceptional shift every 10 sweeps without deflation)
  {
    int hi = s - 1, sweeps = 0, total = 0;
    const double eps = 2.220446049250313e-16;
    while (hi > 0) {
      int l = hi;
      while (l > 0) {
        const double sub = cabs_(A2[(l - 1) * kRcLd + l]);
        const double dia = cabs_(A2[(l - 1) * kRcLd + l - 1]) + cabs_(A2[l * kRcLd + l]);
        if (sub <= eps * dia || sub < 1e-300) break;
        --l;
      }
      __syncthreads();
      if (l == hi) {
        if (tid == 0 && hi > 0) A2[(hi - 1) * kRcLd + hi] = zero;
        __syncthreads();
        --hi;
        sweeps = 0;
        continue;
      }
      if (l > 0) {
        if (tid == 0) A2[(l - 1) * kRcLd + l] = zero;
        __syncthreads();
      }
      if (++total > 60 * s) {
        if (tid == 0) info[0] = 1;
        return;
      }
      ++sweeps;
      // shift: eigenvalue of the trailing 2x2 closer to its last entry
      const double2 a = A2[(hi - 1) * kRcLd + hi - 1], b = A2[hi * kRcLd + hi - 1];
      const double2 cc = A2[(hi - 1) * kRcLd + hi], d = A2[hi * kRcLd + hi];
      double2 shift;
      if (sweeps % 10 == 0) {
        shift = cadd(d, make_double2(cabs_(cc) * 0.75, 0.0));
      } else {
        const double2 tr2 = cscale(cadd(a, d), 0.5);
        const double2 hd = cscale(csub(a, d), 0.5);
        const double2 disc = csqrt_(cadd(cmul(hd, hd), cmul(b, cc)));
        const double2 e1 = cadd(tr2, disc), e2 = csub(tr2, disc);
        shift = cabs2(csub(e1, d)) <= cabs2(csub(e2, d)) ? e1 : e2;
      }
      double2 x = csub(A2[l * kRcLd + l], shift);
      double2 y = A2[l * kRcLd + l + 1];
      for (int r = l; r < hi; ++r) {
        if (r > l) {
          x = A2[(r - 1) * kRcLd + r];
          y = A2[(r - 1) * kRcLd + r + 1];
        }
        double c;
        double2 sn;
        givens_cs(x, y, c, sn);
        __syncthreads();
        rot_rows(A2, r, r > l ? r - 1 : l, s, c, sn);
        __syncthreads();
        rot_cols(A2, r, 0, min(r + 3, hi + 1), c, sn);
        rot_cols(A1, r, 0, s, c, sn);
        __syncthreads();
        if (r > l && tid == 0) A2[(r - 1) * kRcLd + r + 1] = zero;
        __syncthreads();
      }
    }
  }
  __syncthreads();

  // select the knew eigenvalues 1/theta of largest modulus and move them,
  // in that order, to the front of the Schur form by adjacent swaps
  for (int t = 0; t < knew; ++t) {
    if (tid == 0) {
      int best = t;
      double bm = -1.0;
      for (int i = t; i < s; ++i) {
        const double m2 = cabs2(A2[i * kRcLd + i]);
        if (m2 > bm) {
          bm = m2;
          best = i;
        }
      }
      sel[0] = best;
    }
    __syncthreads();
    for (int r = sel[0] - 1; r >= t; --r) {
      // swap the diagonal entries r, r+1: rotation that maps the eigenvector
      // of T[r+1][r+1] within the 2x2 block to e_r
      const double2 t11 = A2[r * kRcLd + r], t22 = A2[(r + 1) * kRcLd + r + 1];
      const double2 t12 = A2[(r + 1) * kRcLd + r];
      double c;
      double2 sn;
      givens_cs(t12, csub(t22, t11), c, sn);
      __syncthreads();
      rot_rows(A2, r, r, s, c, sn);
      __syncthreads();
      rot_cols(A2, r, 0, r + 2, c, sn);
      rot_cols(A1, r, 0, s, c, sn);
      __syncthreads();
      if (tid == 0) {
        A2[r * kRcLd + r + 1] = zero;
        A2[r * kRcLd + r] = t22;
        A2[(r + 1) * kRcLd + r + 1] = t11;
      }
      __syncthreads();
    }
    __syncthreads();   // every thread has read sel[0] before it changes
  }
  for (int i = tid; i < s; i += blockDim.x) mu[i] = A2[i * kRcLd + i];
  __syncthreads();

  // Gbar P (rows x knew), P = leading knew Schur vectors (columns of A1)
  for (int e = tid; e < knew * kRcLd; e += blockDim.x) {
    const int q = e / kRcLd, i = e % kRcLd;
    double2 acc = zero;
    if (i < rows) {
      for (int l = 0; l < s; ++l) {
        double2 g;
        if (l < kk) g = (i == l) ? make_double2(dsc[l], 0.0) : zero;
        else g = G[(int64_t)l * kRcLd + i];
        acc = cadd(acc, cmul(g, A1[q * kRcLd + l]));
      }
    }
    A2[q * kRcLd + i] = acc;
  }
  for (int e = tid; e < kRcK * kRcK; e += blockDim.x) Rk[e] = zero;
  __syncthreads();
  // Gbar P = Qk Rk by Gram-Schmidt with one reorthogonalisation, in place
  for (int q = 0; q < knew; ++q) {
    for (int pass = 0; pass < 2; ++pass) {
      // coefficients against the previous columns, one thread per column
      if (tid < q) {
        double2 d = zero;
        for (int i = 0; i < rows; ++i) d = cadd(d, conj_mul(A2[tid * kRcLd + i], A2[q * kRcLd + i]));
        vh[tid] = d;
      }
      __syncthreads();
      for (int i = tid; i < rows; i += blockDim.x) {
        double2 v = A2[q * kRcLd + i];
        for (int l = 0; l < q; ++l) v = csub(v, cmul(A2[l * kRcLd + i], vh[l]));
        A2[q * kRcLd + i] = v;
      }
      if (tid < q) Rk[q * kRcK + tid] = cadd(Rk[q * kRcK + tid], vh[tid]);
      __syncthreads();
    }
    double part = 0.0;
    for (int i = tid; i < rows; i += blockDim.x) part += cabs2(A2[q * kRcLd + i]);
    const double nrm = sqrt(block_sum(part, red));
    if (!(nrm > 0.0)) {
      if (tid == 0) info[0] = 1;
      return;
    }
    for (int i = tid; i < rows; i += blockDim.x) A2[q * kRcLd + i] = cscale(A2[q * kRcLd + i], 1.0 / nrm);
    if (tid == 0) Rk[q * kRcK + q] = make_double2(nrm, 0.0);
    __syncthreads();
  }
  // Mc = Qk
  for (int e = tid; e < knew * kRcLd; e += blockDim.x) {
    const int q = e / kRcLd, i = e % kRcLd;
    Mc[(int64_t)q * kRcLd + i] = (i < rows) ? A2[q * kRcLd + i] : zero;
  }
  __syncthreads();
  // Mu = P Rk^{-1}: row i solves x Rk = p_i by forward substitution (kept in
  // row i of A2, which only thread i touches); D folded into rows < kk
  for (int i = tid; i < kRcLd; i += blockDim.x) {
    const double di = i < kk ? dsc[i] : 1.0;
    for (int q = 0; q < knew; ++q) {
      double2 v = zero;
      if (i < s) {
        double2 t = A1[q * kRcLd + i];
        for (int l = 0; l < q; ++l) t = csub(t, cmul(A2[l * kRcLd + i], Rk[q * kRcK + l]));
        v = cdiv(t, Rk[q * kRcK + q]);
      }
      A2[q * kRcLd + i] = v;
      Mu[(int64_t)q * kRcLd + i] = cscale(v, di);
    }
  }
  if (tid == 0) info[0] = 0;
}

void launch_rc_save(hipStream_t st, int kk, int j, const double2* h, const double* hn, double2* G) {
  hipLaunchKernelGGL(k_rc_save, dim3(1), dim3(128), 0, st, kk, j, h, hn, G);
}

void launch_rc_by(hipStream_t st, int kk, const int* jd, const double2* G, const double2* y, double2* t) {
  hipLaunchKernelGGL(k_rc_by, dim3(1), dim3(64), 0, st, kk, jd, G, y, t);
}

void launch_rc_ritz(hipStream_t st, int kk, int jd, int knew, int extra, int ldw, const double2* G,
                    const double2* WVg, const double2* UU, double2* Mc, double2* Mu, double2* mu, int* info) {
  hipLaunchKernelGGL(k_rc_ritz, dim3(1), dim3(256), 0, st, kk, jd, knew, extra, ldw, G, WVg, UU, Mc, Mu, mu, info);
}

// Block cycles (p right-hand sides): columns kk + j p .. kk + (j+1) p - 1 of
// Gbar from block step j: rows < kk the coefficients against C (B1 + B2, two
// Gram-Schmidt passes, ld kk), rows kk .. kk + (j+1) p - 1 those against
// the previous blocks (H1 + H2, ld (j+1) p), the next p rows the new block's
// triangular factor S (p x p), the rest zero.
__global__ void k_rc_save_block(int kk, int j, int p, const double2* __restrict__ B1, const double2* __restrict__ B2,
                                const double2* __restrict__ H1, const double2* __restrict__ H2,
                                const double2* __restrict__ S, double2* __restrict__ G) {
  const int c = blockIdx.x;   // column of the block step, < p
  const int q = (j + 1) * p;
  for (int i = threadIdx.x; i < kRcLd; i += blockDim.x) {
    double2 v = make_double2(0.0, 0.0);
    if (i < kk) {
      v = cadd(B1[(int64_t)c * kk + i], B2[(int64_t)c * kk + i]);
    } else if (i < kk + q) {
      const int r = i - kk;
      v = cadd(H1[(int64_t)c * q + r], H2[(int64_t)c * q + r]);
    } else if (i < kk + q + p) {
      v = S[(int64_t)c * p + (i - kk - q)];
    }
    G[(int64_t)(kk + j * p + c) * kRcLd + i] = v;
  }
}

void launch_rc_save_block(hipStream_t st, int kk, int j, int p, const double2* B1, const double2* B2,
                          const double2* H1, const double2* H2, const double2* S, double2* G) {
  hipLaunchKernelGGL(k_rc_save_block, dim3(p), dim3(64), 0, st, kk, j, p, B1, B2, H1, H2, S, G);
}

// T (kk x p, ld kk) = -B Y: the recycled part of a block cycle's update;
// B = rows < kk of Gbar's columns kk .. kk + q - 1, Y (q x p, ld ldy).
__global__ void k_rc_by_block(int kk, int q, int p, const double2* __restrict__ G, const double2* __restrict__ Y,
                              int ldy, double2* __restrict__ T) {
  const int c = blockIdx.x, i = threadIdx.x;
  if (i >= kk) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int l = 0; l < q; ++l) acc = cadd(acc, cmul(G[(int64_t)(kk + l) * kRcLd + i], Y[(int64_t)c * ldy + l]));
  T[(int64_t)c * kk + i] = make_double2(-acc.x, -acc.y);
}

void launch_rc_by_block(hipStream_t st, int kk, int q, int p, const double2* G, const double2* Y, int ldy,
                        double2* T) {
  if (kk > 0) hipLaunchKernelGGL(k_rc_by_block, dim3(p), dim3(64), 0, st, kk, q, p, G, Y, ldy, T);
}

}  // namespace mxw
