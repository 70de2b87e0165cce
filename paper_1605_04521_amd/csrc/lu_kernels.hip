// Batched dense complex LU with partial pivoting of the subdomain matrices A_s
// (the factorised local solves A_s^{-1} of ORAS, Sec. 4), in FP64 or FP32.
//
// Storage per subdomain: column-major, leading dimension ld, real plane then
// imaginary plane.  One workgroup (4 wavefronts) factorises one matrix with a
// right-looking blocked algorithm of panel width NB:
//   1. panel: unblocked LU of columns [k, k+NB) with pivot search on
//      |re| + |im| (lowest row on ties), row swaps inside the panel;
//   2. the panel's row interchanges are applied to the other columns as one
//      net permutation of the affected rows;
//   3. L11^{-1} (unit lower) and U11^{-1} are formed; U12 = L11^{-1} A12 and
//      A22 -= L21 U12 run as complex GEMMs on MFMA (4 real products each);
//   4. the diagonal block is replaced by [L11^{-1} strict lower | U11^{-1}],
//      which turns the diagonal solves of the triangular sweeps into products.
// perm receives the row permutation: (P A)[i] = A[perm[i]].
#include "device.h"
#include "kernels.h"

namespace mxw {

constexpr int kPad = 4;

template <typename R, int NB>
struct LuSmem {
  R Are[NB][64 + kPad];
  R Aim[NB][64 + kPad];
  R Bre[NB][64 + kPad];
  R Bim[NB][64 + kPad];
  double rv[256];
  int ri[256];
  R ur[NB], ui[NB];
  int piv[NB];
  int src[2 * NB], dst[2 * NB];
  int npairs;
};

// C[M x N] = (sub ? C - A B : A B); A is M x NB (lda), B is NB x N (ldb), all
// column-major complex split planes.  The product is formed transposed
// (D = B^T A^T on MFMA) so that each lane's outputs run down a column of C.
template <typename R, int NB>
__device__ void wg_cgemm(int M, int N, const R* __restrict__ Ar, const R* __restrict__ Ai, int64_t lda,
                         const R* Br, const R* Bi, int64_t ldb, R* Cr, R* Ci, int64_t ldc, bool sub,
                         LuSmem<R, NB>& sm) {
  typedef typename Mfma<R>::acc_t acc_t;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  for (int n0 = 0; n0 < N; n0 += 64) {
    __syncthreads();
    for (int idx = tid; idx < NB * 64; idx += 256) {
      const int kk = idx % NB, cc = idx / NB, c = n0 + cc;
      R vr = R(0), vi = R(0);
      if (c < N) {
        vr = Br[(int64_t)c * ldb + kk];
        vi = Bi[(int64_t)c * ldb + kk];
      }
      sm.Bre[kk][cc] = vr;
      sm.Bim[kk][cc] = vi;
    }
    for (int m0 = 0; m0 < M; m0 += 64) {
      for (int idx = tid; idx < 64 * NB; idx += 256) {
        const int rr = idx & 63, kk = idx >> 6, r = m0 + rr;
        R vr = R(0), vi = R(0);
        if (r < M) {
          vr = Ar[(int64_t)kk * lda + r];
          vi = Ai[(int64_t)kk * lda + r];
        }
        sm.Are[kk][rr] = vr;
        sm.Aim[kk][rr] = vi;
      }
      __syncthreads();
      acc_t dre[2][2], dim[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          dre[a][b] = acc_t{0, 0, 0, 0};
          dim[a][b] = acc_t{0, 0, 0, 0};
        }
#pragma unroll 4
      for (int k0 = 0; k0 < NB; k0 += 4) {
        const int kk = k0 + lk;
        R bre[2], bim[2], are[2], aim[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          bre[c] = sm.Bre[kk][wc * 32 + c * 16 + li];
          bim[c] = sm.Bim[kk][wc * 32 + c * 16 + li];
          are[c] = sm.Are[kk][wr * 32 + c * 16 + li];
          aim[c] = sm.Aim[kk][wr * 32 + c * 16 + li];
        }
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            dre[c][r] = Mfma<R>::op(bre[c], are[r], dre[c][r]);
            dre[c][r] = Mfma<R>::op(-bim[c], aim[r], dre[c][r]);
            dim[c][r] = Mfma<R>::op(bre[c], aim[r], dim[c][r]);
            dim[c][r] = Mfma<R>::op(bim[c], are[r], dim[c][r]);
          }
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int col = n0 + wc * 32 + c * 16 + Mfma<R>::row(lane, v);
            const int row = m0 + wr * 32 + r * 16 + li;
            if (row < M && col < N) {
              const int64_t o = (int64_t)col * ldc + row;
              if (sub) {
                Cr[o] -= dre[c][r][v];
                Ci[o] -= dim[c][r][v];
              } else {
                Cr[o] = dre[c][r][v];
                Ci[o] = dim[c][r][v];
              }
            }
          }
      __syncthreads();
    }
  }
}

template <typename R, int NB>
__global__ void __launch_bounds__(256) k_lu(R* __restrict__ F, const int64_t* __restrict__ foff,
                                            const int* __restrict__ nsz, const int* __restrict__ lds,
                                            int* __restrict__ perm, const int64_t* __restrict__ poff,
                                            R* __restrict__ scratch, int* __restrict__ info,
                                            const int* __restrict__ order) {
  __shared__ LuSmem<R, NB> sm;
  const int s = order ? order[blockIdx.x] : blockIdx.x;
  const int n = nsz[s];
  const int64_t ld = lds[s];
  R* Ar = F + foff[s];
  R* Ai = Ar + ld * n;
  int* P = perm + poff[s];
  R* Wr = scratch + (int64_t)blockIdx.x * 2 * NB * NB;   // L11^{-1}, NB x NB
  R* Wi = Wr + NB * NB;
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += 256) P[i] = i;
  int first_zero = 0;
  // singularity threshold: |pivot| <= n u max|A_s| (FP64) or u max|A_s| (FP32)
  double amax = 0.0;
  for (int c = 0; c < n; ++c)
    for (int i = tid; i < n; i += 256)
      amax = fmax(amax, fabs((double)Ar[(int64_t)c * ld + i]) + fabs((double)Ai[(int64_t)c * ld + i]));
  sm.rv[tid] = amax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) sm.rv[tid] = fmax(sm.rv[tid], sm.rv[tid + w]);
    __syncthreads();
  }
  const double tiny = (sizeof(R) == 8 ? (double)n * 2.220446049250313e-16 : 1.1920928955078125e-07) * sm.rv[0];
  __syncthreads();

  for (int k = 0; k < n; k += NB) {
    const int kb = min(NB, n - k);
    // ---- 1. panel factorisation
    for (int jj = 0; jj < kb; ++jj) {
      const int j = k + jj;
      const R* cr = Ar + (int64_t)j * ld;
      const R* ci = Ai + (int64_t)j * ld;
      double best = -1.0;
      int bi = 0x7fffffff;
      for (int i = j + tid; i < n; i += 256) {
        const double v = fabs((double)cr[i]) + fabs((double)ci[i]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      sm.rv[tid] = best;
      sm.ri[tid] = bi;
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
          const double o = sm.rv[tid + w];
          const int oi = sm.ri[tid + w];
          if (o > sm.rv[tid] || (o == sm.rv[tid] && oi < sm.ri[tid])) {
            sm.rv[tid] = o;
            sm.ri[tid] = oi;
          }
        }
        __syncthreads();
      }
      const int p = sm.ri[0];
      const bool zero = !(sm.rv[0] > tiny);
      if (zero && first_zero == 0) first_zero = j + 1;
      if (p != j && tid < kb) {
        const int64_t c = (int64_t)(k + tid) * ld;
        R t0 = Ar[c + j], t1 = Ai[c + j];
        Ar[c + j] = Ar[c + p];
        Ai[c + j] = Ai[c + p];
        Ar[c + p] = t0;
        Ai[c + p] = t1;
      }
      if (tid == 0) sm.piv[jj] = p;
      __syncthreads();
      if (tid < kb) {
        sm.ur[tid] = Ar[(int64_t)(k + tid) * ld + j];
        sm.ui[tid] = Ai[(int64_t)(k + tid) * ld + j];
      }
      __syncthreads();
      const R pr = sm.ur[jj], pi = sm.ui[jj];
      const R den = pr * pr + pi * pi;
      const R rr = den > R(0) ? pr / den : R(0), ri = den > R(0) ? -pi / den : R(0);
      for (int i = j + 1 + tid; i < n; i += 256) {
        const R ar = Ar[(int64_t)j * ld + i], ai = Ai[(int64_t)j * ld + i];
        const R lr = ar * rr - ai * ri, lim = ar * ri + ai * rr;
        Ar[(int64_t)j * ld + i] = lr;
        Ai[(int64_t)j * ld + i] = lim;
        for (int c = jj + 1; c < kb; ++c) {
          const int64_t o = (int64_t)(k + c) * ld + i;
          const R ur = sm.ur[c], ui = sm.ui[c];
          Ar[o] -= lr * ur - lim * ui;
          Ai[o] -= lr * ui + lim * ur;
        }
      }
      __syncthreads();
    }
    // ---- 2. net row permutation of the panel's interchanges
    if (tid == 0) {
      int rows[2 * NB], cont[2 * NB], m = 0;
      for (int jj = 0; jj < kb; ++jj) {
        rows[m] = k + jj;
        cont[m] = k + jj;
        ++m;
      }
      for (int jj = 0; jj < kb; ++jj) {
        const int p = sm.piv[jj];
        int found = -1;
        for (int q = 0; q < m; ++q)
          if (rows[q] == p) found = q;
        if (found < 0) {
          rows[m] = p;
          cont[m] = p;
          found = m++;
        }
        const int a = jj;   // rows[jj] == k + jj
        const int t = cont[a];
        cont[a] = cont[found];
        cont[found] = t;
        const int tp = P[k + jj];
        P[k + jj] = P[p];
        P[p] = tp;
      }
      int np = 0;
      for (int q = 0; q < m; ++q)
        if (cont[q] != rows[q]) {
          sm.dst[np] = rows[q];
          sm.src[np] = cont[q];
          ++np;
        }
      sm.npairs = np;
    }
    __syncthreads();
    {
      const int np = sm.npairs;
      const int lane = tid & 63, wave = tid >> 6;
      if (np > 0) {
        for (int c = wave; c < n; c += 4) {
          if (c >= k && c < k + kb) continue;
          R vr = R(0), vi = R(0);
          if (lane < np) {
            vr = Ar[(int64_t)c * ld + sm.src[lane]];
            vi = Ai[(int64_t)c * ld + sm.src[lane]];
          }
          __builtin_amdgcn_wave_barrier();
          if (lane < np) {
            Ar[(int64_t)c * ld + sm.dst[lane]] = vr;
            Ai[(int64_t)c * ld + sm.dst[lane]] = vi;
          }
        }
      }
    }
    __syncthreads();
    // ---- 3. inverses of the diagonal block factors
    for (int idx = tid; idx < kb * kb; idx += 256) {
      const int i = idx % kb, c = idx / kb;
      sm.Are[c][i] = Ar[(int64_t)(k + c) * ld + k + i];
      sm.Aim[c][i] = Ai[(int64_t)(k + c) * ld + k + i];
    }
    __syncthreads();
    if (tid < kb) {
      // column c of L11^{-1}: x_c = 1, x_i = -sum_{c<=m<i} L[i][m] x_m
      const int c = tid;
      for (int i = 0; i < NB; ++i) {
        R xr = R(0), xi = R(0);
        if (i == c) xr = R(1);
        if (i > c && i < kb) {
          for (int m = c; m < i; ++m) {
            const R lr = sm.Are[m][i], lim = sm.Aim[m][i];
            const R yr = (m == c) ? R(1) : Wr[c * NB + m], yi = (m == c) ? R(0) : Wi[c * NB + m];
            xr -= lr * yr - lim * yi;
            xi -= lr * yi + lim * yr;
          }
        }
        Wr[c * NB + i] = xr;
        Wi[c * NB + i] = xi;
      }
    } else if (tid >= 64 && tid < 64 + kb) {
      // column c of U11^{-1}: x_c = 1/U_cc, x_i = -(sum_{i<m<=c} U[i][m] x_m)/U_ii
      const int c = tid - 64;
      R xr[NB], xi[NB];
      for (int i = 0; i < NB; ++i) xr[i] = xi[i] = R(0);
      for (int i = c; i >= 0; --i) {
        R sr = (i == c) ? R(1) : R(0), si = R(0);
        for (int m = i + 1; m <= c; ++m) {
          const R ur = sm.Are[m][i], ui = sm.Aim[m][i];
          sr -= ur * xr[m] - ui * xi[m];
          si -= ur * xi[m] + ui * xr[m];
        }
        const R dr = sm.Are[i][i], di = sm.Aim[i][i];
        const R den = dr * dr + di * di;
        const R ir = den > R(0) ? dr / den : R(0), ii = den > R(0) ? -di / den : R(0);
        xr[i] = sr * ir - si * ii;
        xi[i] = sr * ii + si * ir;
      }
      for (int i = 0; i < NB; ++i) {
        sm.Bre[c][i] = xr[i];
        sm.Bim[c][i] = xi[i];
      }
    }
    __syncthreads();
    for (int idx = tid; idx < kb * kb; idx += 256) {
      const int i = idx % kb, c = idx / kb;
      const int64_t o = (int64_t)(k + c) * ld + k + i;
      if (i > c) {
        Ar[o] = Wr[c * NB + i];
        Ai[o] = Wi[c * NB + i];
      } else {
        Ar[o] = sm.Bre[c][i];
        Ai[o] = sm.Bim[c][i];
      }
    }
    __syncthreads();
    const int nt = n - k - kb;
    if (nt > 0) {
      // U12 = L11^{-1} A12 (in place), then A22 -= L21 U12
      R* A12r = Ar + (int64_t)(k + kb) * ld + k;
      R* A12i = Ai + (int64_t)(k + kb) * ld + k;
      wg_cgemm<R, NB>(kb, nt, Wr, Wi, NB, A12r, A12i, ld, A12r, A12i, ld, false, sm);
      __syncthreads();
      const R* L21r = Ar + (int64_t)k * ld + k + kb;
      const R* L21i = Ai + (int64_t)k * ld + k + kb;
      R* A22r = Ar + (int64_t)(k + kb) * ld + k + kb;
      R* A22i = Ai + (int64_t)(k + kb) * ld + k + kb;
      wg_cgemm<R, NB>(nt, nt, L21r, L21i, ld, A12r, A12i, ld, A22r, A22i, ld, true, sm);
      __syncthreads();
    }
  }
  if (tid == 0) info[s] = first_zero;
}

template <typename R>
void launch_lu(hipStream_t st, int n_sub, R* F, const int64_t* foff, const int* nsz, const int* lds, int* perm,
               const int64_t* poff, R* scratch, int* info, const int* order) {
  if (n_sub > 0)
    hipLaunchKernelGGL((k_lu<R, kLuNB>), dim3(n_sub), dim3(256), 0, st, F, foff, nsz, lds, perm, poff, scratch, info,
                       order);
}
template void launch_lu<double>(hipStream_t, int, double*, const int64_t*, const int*, const int*, int*,
                                const int64_t*, double*, int*, const int*);
template void launch_lu<float>(hipStream_t, int, float*, const int64_t*, const int*, const int*, int*,
                               const int64_t*, float*, int*, const int*);

}  // namespace mxw
