// Batched dense complex LU with partial pivoting of the subdomain matrices A_s
// (the factorised local solves A_s^{-1} of ORAS, Sec. 4), in FP64 or FP32.
//
// Storage per subdomain: column-major, leading dimension ld, real plane then
// imaginary plane.  One workgroup (4 wavefronts) factorises one matrix with a
// right-looking blocked algorithm of panel width NB:
//   1. panel: unblocked LU of columns [k, k+NB) with pivot search on
//      |re| + |im| (lowest row on ties); the search for the next column is
//      fused into the rank-1 update of the current one;
//   2. the panel's row interchanges are applied to the other columns as one
//      net permutation of the affected rows;
//   3. L11^{-1} (unit lower) and U11^{-1} are formed in LDS; U12 = L11^{-1} A12
//      and A22 -= L21 U12 run as complex GEMMs on MFMA (4 real products each),
//      accumulating straight into the C tile held in the MFMA accumulators;
//   4. the diagonal block is replaced by [L11^{-1} strict lower | U11^{-1}],
//      which turns the diagonal solves of the triangular sweeps into products.
// perm receives the row permutation: (P A)[i] = A[perm[i]].
#include "device.h"
#include "kernels.h"

namespace mxw {

constexpr int kPad = 4;

template <typename R, int NB>
struct LuSmem {
  // GEMM tiles: A tile [k][row], B tile [k][col].  While the diagonal block
  // is inverted, Are/Aim[c][0..NB) hold its copy (column c) and
  // Are/Aim[c][NB..2NB) column c of L11^{-1}; Bre/Bim[c][0..NB) column c of U11^{-1}.
  R Are[NB][64 + kPad];
  R Aim[NB][64 + kPad];
  R Bre[NB][64 + kPad];
  R Bim[NB][64 + kPad];
  double rv[4];
  int ri[4];
  R ur[NB], ui[NB];
  int piv[NB];
  int src[2 * NB], dst[2 * NB];
  int rows[2 * NB], cont[2 * NB];
  int npairs;
};

__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(i, o, 64);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

// C[M x N] = (sub ? C - A B : A B); A is M x NB (lda), B is NB x N (ldb), all
// column-major complex split planes.  The product is formed transposed
// (D = B^T A^T on MFMA) so that each lane's outputs run down a column of C;
// the accumulators start from C (sub) and B enters with the sign folded in.
template <typename R, int NB>
__device__ void wg_cgemm(int M, int N, const R* __restrict__ Ar, const R* __restrict__ Ai, int64_t lda,
                         const R* Br, const R* Bi, int64_t ldb, R* Cr, R* Ci, int64_t ldc, bool sub,
                         LuSmem<R, NB>& sm) {
  typedef typename Mfma<R>::acc_t acc_t;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const R sgn = sub ? R(-1) : R(1);
  for (int n0 = 0; n0 < N; n0 += 64) {
    __syncthreads();
    for (int idx = tid; idx < NB * 64; idx += 256) {
      const int kk = idx % NB, cc = idx / NB, c = n0 + cc;
      R vr = R(0), vi = R(0);
      if (c < N) {
        vr = sgn * Br[(int64_t)c * ldb + kk];
        vi = sgn * Bi[(int64_t)c * ldb + kk];
      }
      sm.Bre[kk][cc] = vr;
      sm.Bim[kk][cc] = vi;
    }
    for (int m0 = 0; m0 < M; m0 += 64) {
      acc_t dre[2][2], dim[2][2];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int col = n0 + wc * 32 + c * 16 + Mfma<R>::row(lane, v);
            const int row = m0 + wr * 32 + r * 16 + li;
            R a = R(0), b = R(0);
            if (sub && row < M && col < N) {
              a = Cr[(int64_t)col * ldc + row];
              b = Ci[(int64_t)col * ldc + row];
            }
            dre[c][r][v] = a;
            dim[c][r][v] = b;
          }
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
#pragma unroll 2
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
              Cr[(int64_t)col * ldc + row] = dre[c][r][v];
              Ci[(int64_t)col * ldc + row] = dim[c][r][v];
            }
          }
      __syncthreads();
    }
  }
}

template <typename R, int NB>
__global__ void __launch_bounds__(256, 2) k_lu(R* __restrict__ F, const int64_t* __restrict__ foff,
                                               const int* __restrict__ nsz, const int* __restrict__ lds,
                                               int* __restrict__ perm, const int64_t* __restrict__ poff,
                                               R* __restrict__ scratch, int* __restrict__ info,
                                               const int* __restrict__ order) {
  static_assert(2 * NB <= 64 + kPad, "inverse workspace must fit the tile rows");
  __shared__ LuSmem<R, NB> sm;
  const int s = order ? order[blockIdx.x] : blockIdx.x;
  const int n = nsz[s];
  const int64_t ld = lds[s];
  R* Ar = F + foff[s];
  R* Ai = Ar + ld * n;
  int* P = perm + poff[s];
  R* Wr = scratch + (int64_t)blockIdx.x * 2 * NB * NB;   // L11^{-1} (unit lower, full NB x NB)
  R* Wi = Wr + NB * NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < n; i += 256) P[i] = i;
  int first_zero = 0;
  // singularity threshold: |pivot| <= n u max|A_s| (FP64) or u max|A_s| (FP32)
  double tiny;
  {
    double amax = 0.0;
    for (int c = 0; c < n; ++c)
      for (int i = tid; i < n; i += 256)
        amax = fmax(amax, fabs((double)Ar[(int64_t)c * ld + i]) + fabs((double)Ai[(int64_t)c * ld + i]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
    if (lane == 0) sm.rv[wave] = amax;
    __syncthreads();
    amax = fmax(fmax(sm.rv[0], sm.rv[1]), fmax(sm.rv[2], sm.rv[3]));
    tiny = (sizeof(R) == 8 ? (double)n * 2.220446049250313e-16 : 1.1920928955078125e-07) * amax;
    __syncthreads();
  }

  for (int k = 0; k < n; k += NB) {
    const int kb = min(NB, n - k);
    // ---- 1. panel factorisation; (best, bi): this thread's candidate pivot
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = k + tid; i < n; i += 256) {
      const double v = fabs((double)Ar[(int64_t)k * ld + i]) + fabs((double)Ai[(int64_t)k * ld + i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int jj = 0; jj < kb; ++jj) {
      const int j = k + jj;
      wave_argmax(best, bi);
      if (lane == 0) {
        sm.rv[wave] = best;
        sm.ri[wave] = bi;
      }
      __syncthreads();
      double pv = sm.rv[0];
      int p = sm.ri[0];
#pragma unroll
      for (int w = 1; w < 4; ++w)
        if (sm.rv[w] > pv || (sm.rv[w] == pv && sm.ri[w] < p)) {
          pv = sm.rv[w];
          p = sm.ri[w];
        }
      if (!(pv > tiny) && first_zero == 0) first_zero = j + 1;
      if (p < j || p >= n) p = j;   // all candidates empty (cannot happen for j < n)
      if (p != j && tid < kb) {
        const int64_t c = (int64_t)(k + tid) * ld;
        const R t0 = Ar[c + j], t1 = Ai[c + j];
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
      best = -1.0;
      bi = 0x7fffffff;
      for (int i = j + 1 + tid; i < n; i += 256) {
        const R ar = Ar[(int64_t)j * ld + i], ai = Ai[(int64_t)j * ld + i];
        const R lr = ar * rr - ai * ri, lim = ar * ri + ai * rr;
        Ar[(int64_t)j * ld + i] = lr;
        Ai[(int64_t)j * ld + i] = lim;
        for (int c = jj + 1; c < kb; ++c) {
          const int64_t o = (int64_t)(k + c) * ld + i;
          const R nr = Ar[o] - (lr * sm.ur[c] - lim * sm.ui[c]);
          const R ni = Ai[o] - (lr * sm.ui[c] + lim * sm.ur[c]);
          Ar[o] = nr;
          Ai[o] = ni;
          if (c == jj + 1) {
            const double v = fabs((double)nr) + fabs((double)ni);
            if (v > best) {
              best = v;
              bi = i;
            }
          }
        }
      }
    }
    // ---- 2. net row permutation of the panel's interchanges
    if (tid == 0) {
      int* rows = sm.rows;
      int* cont = sm.cont;
      int m = 0;
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
        const int t = cont[jj];
        cont[jj] = cont[found];
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
      if (np > 0) {
        const int sr = lane < np ? sm.src[lane] : 0, ds = lane < np ? sm.dst[lane] : 0;
        for (int c0 = wave * 4; c0 < n; c0 += 16) {
          R vr[4], vi[4];
          bool ok[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int c = c0 + u;
            ok[u] = lane < np && c < n && (c < k || c >= k + kb);
            vr[u] = ok[u] ? Ar[(int64_t)c * ld + sr] : R(0);
            vi[u] = ok[u] ? Ai[(int64_t)c * ld + sr] : R(0);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (ok[u]) {
              Ar[(int64_t)(c0 + u) * ld + ds] = vr[u];
              Ai[(int64_t)(c0 + u) * ld + ds] = vi[u];
            }
        }
      }
    }
    // ---- 3. inverses of the diagonal block factors (in LDS)
    for (int idx = tid; idx < kb * kb; idx += 256) {
      const int i = idx % kb, c = idx / kb;
      sm.Are[c][i] = Ar[(int64_t)(k + c) * ld + k + i];
      sm.Aim[c][i] = Ai[(int64_t)(k + c) * ld + k + i];
    }
    __syncthreads();
    if (tid < kb) {
      // column c of L11^{-1}: x_c = 1, x_i = -sum_{c<=m<i} L[i][m] x_m
      const int c = tid;
      for (int i = 0; i < kb; ++i) {
        R xr = (i == c) ? R(1) : R(0), xi = R(0);
        if (i > c) {
          for (int m = c; m < i; ++m) {
            const R lr = sm.Are[m][i], lim = sm.Aim[m][i];
            const R yr = (m == c) ? R(1) : sm.Are[c][NB + m], yi = (m == c) ? R(0) : sm.Aim[c][NB + m];
            xr -= lr * yr - lim * yi;
            xi -= lr * yi + lim * yr;
          }
        }
        sm.Are[c][NB + i] = xr;
        sm.Aim[c][NB + i] = xi;
      }
    } else if (tid >= 64 && tid < 64 + kb) {
      // column c of U11^{-1}: x_i = (delta_ic - sum_{i<m<=c} U[i][m] x_m) / U_ii
      const int c = tid - 64;
      for (int i = c + 1; i < kb; ++i) {
        sm.Bre[c][i] = R(0);
        sm.Bim[c][i] = R(0);
      }
      for (int i = c; i >= 0; --i) {
        R sr = (i == c) ? R(1) : R(0), si = R(0);
        for (int m = i + 1; m <= c; ++m) {
          const R ur = sm.Are[m][i], ui = sm.Aim[m][i];
          const R xr = sm.Bre[c][m], xi = sm.Bim[c][m];
          sr -= ur * xr - ui * xi;
          si -= ur * xi + ui * xr;
        }
        const R dr = sm.Are[i][i], di = sm.Aim[i][i];
        const R den = dr * dr + di * di;
        const R ir = den > R(0) ? dr / den : R(0), ii = den > R(0) ? -di / den : R(0);
        sm.Bre[c][i] = sr * ir - si * ii;
        sm.Bim[c][i] = sr * ii + si * ir;
      }
    }
    __syncthreads();
    for (int idx = tid; idx < NB * NB; idx += 256) {
      const int i = idx % NB, c = idx / NB;
      const bool in = i < kb && c < kb;
      if (in) {
        const int64_t o = (int64_t)(k + c) * ld + k + i;
        if (i > c) {
          Ar[o] = sm.Are[c][NB + i];
          Ai[o] = sm.Aim[c][NB + i];
        } else {
          Ar[o] = sm.Bre[c][i];
          Ai[o] = sm.Bim[c][i];
        }
      }
      Wr[c * NB + i] = (in && i >= c) ? sm.Are[c][NB + i] : R(0);
      Wi[c * NB + i] = (in && i >= c) ? sm.Aim[c][NB + i] : R(0);
    }
    __syncthreads();
    const int nt = n - k - kb;
    if (nt > 0) {
      // U12 = L11^{-1} A12 (in place), then A22 -= L21 U12
      R* A12r = Ar + (int64_t)(k + kb) * ld + k;
      R* A12i = Ai + (int64_t)(k + kb) * ld + k;
      wg_cgemm<R, NB>(kb, nt, Wr, Wi, NB, A12r, A12i, ld, A12r, A12i, ld, false, sm);
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
    timed_launch(k_lu<R, kLuNB>, dim3(n_sub), dim3(256), 0, st, F, foff, nsz, lds, perm, poff, scratch, info,
                 order);
}
template void launch_lu<double>(hipStream_t, int, double*, const int64_t*, const int*, const int*, int*,
                                const int64_t*, double*, int*, const int*);
template void launch_lu<float>(hipStream_t, int, float*, const int64_t*, const int*, const int*, int*,
                               const int64_t*, float*, int*, const int*);

}  // namespace mxw
