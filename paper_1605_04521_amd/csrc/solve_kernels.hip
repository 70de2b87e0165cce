// Per-iteration kernels of preconditioned GMRES (Sec. 4-5):
//   * fused ORAS application: restriction R_s v, row permutation, forward and
//     backward sweeps with the LU factors, Boolean prolongation R_s^T D_s;
//   * complex CSR SpMV (FP64);
//   * classical Gram-Schmidt with reorthogonalisation (two passes) using
//     block partial sums reduced in a fixed order (deterministic);
//   * complex Givens updates of the Hessenberg least-squares problem, the
//     triangular solve for y and the update x += Z y.
// Several right-hand sides run in the same launches (grid dimension y); every
// column keeps its own Krylov space (the pseudo-block scheme of Sec. 5).
#include "device.h"
#include "kernels.h"

namespace mxw {

// ---------------------------------------------------------------------------
// ORAS application, one workgroup per (subdomain, column)
// ---------------------------------------------------------------------------
template <typename R, int NB>
__global__ void __launch_bounds__(256) k_local_solve(const R* __restrict__ F, const int64_t* __restrict__ foff,
                                                     const int* __restrict__ nsz, const int* __restrict__ lds,
                                                     const int* __restrict__ perm, const int64_t* __restrict__ poff,
                                                     const int* __restrict__ sub_dofs, const uint8_t* __restrict__ pou,
                                                     const double2* __restrict__ v, int64_t vstride,
                                                     double2* __restrict__ z, int64_t zstride,
                                                     double2* __restrict__ ys, int64_t ystride,
                                                     const int* __restrict__ active, const int* __restrict__ order) {
  extern __shared__ unsigned char dyn[];
  __shared__ R pr_[8][NB], pi_[8][NB];
  __shared__ R ar_[NB], ai_[NB];
  const int s = order ? order[blockIdx.x] : blockIdx.x;
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int n = nsz[s];
  const int64_t ld = lds[s];
  const R* Ar = F + foff[s];
  const R* Ai = Ar + ld * n;
  const int* P = perm + poff[s];
  const int* D = sub_dofs + poff[s];
  R* xr = reinterpret_cast<R*>(dyn);
  R* xi = xr + n;
  const double2* vc = v + (int64_t)col * vstride;
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += 256) {
    const double2 a = vc[D[P[i]]];
    xr[i] = (R)a.x;
    xi[i] = (R)a.y;
  }
  __syncthreads();
  const int r = tid % NB, cg = tid / NB;   // NB rows x (256/NB) column groups
  constexpr int CG = 256 / NB;
  // forward sweep with unit-lower L; diagonal blocks hold L_kk^{-1}
  for (int b0 = 0; b0 < n; b0 += NB) {
    const int bn = min(NB, n - b0);
    R s0r = 0, s0i = 0, s1r = 0, s1i = 0;
    if (r < bn) {
      const R* cr = Ar + b0 + r;
      const R* ci = Ai + b0 + r;
      int c = cg;
      for (; c + 7 * CG < b0; c += 8 * CG) {
        R lr[8], li[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          lr[u] = cr[(int64_t)(c + u * CG) * ld];
          li[u] = ci[(int64_t)(c + u * CG) * ld];
        }
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          s0r += lr[u] * xr[c + u * CG] - li[u] * xi[c + u * CG];
          s0i += lr[u] * xi[c + u * CG] + li[u] * xr[c + u * CG];
          s1r += lr[u + 1] * xr[c + (u + 1) * CG] - li[u + 1] * xi[c + (u + 1) * CG];
          s1i += lr[u + 1] * xi[c + (u + 1) * CG] + li[u + 1] * xr[c + (u + 1) * CG];
        }
      }
      for (; c < b0; c += CG) {
        const R l0r = cr[(int64_t)c * ld], l0i = ci[(int64_t)c * ld];
        s0r += l0r * xr[c] - l0i * xi[c];
        s0i += l0r * xi[c] + l0i * xr[c];
      }
    }
    pr_[cg][r] = s0r + s1r;
    pi_[cg][r] = s0i + s1i;
    __syncthreads();
    if (tid < bn) {
      R tr = xr[b0 + tid], ti = xi[b0 + tid];
      for (int q = 0; q < CG; ++q) {
        tr -= pr_[q][tid];
        ti -= pi_[q][tid];
      }
      ar_[tid] = tr;
      ai_[tid] = ti;
    }
    __syncthreads();
    R tr = 0, ti = 0;
    if (r < bn) {
      for (int c = cg; c < r; c += CG) {
        const int64_t o = (int64_t)(b0 + c) * ld + b0 + r;
        const R lr = Ar[o], li = Ai[o];
        tr += lr * ar_[c] - li * ai_[c];
        ti += lr * ai_[c] + li * ar_[c];
      }
    }
    pr_[cg][r] = tr;
    pi_[cg][r] = ti;
    __syncthreads();
    if (tid < bn) {
      R yr = ar_[tid], yi = ai_[tid];
      for (int q = 0; q < CG; ++q) {
        yr += pr_[q][tid];
        yi += pi_[q][tid];
      }
      xr[b0 + tid] = yr;
      xi[b0 + tid] = yi;
    }
    __syncthreads();
  }
  // backward sweep with U; diagonal blocks hold U_kk^{-1}
  const int last = ((n - 1) / NB) * NB;
  for (int b0 = last; b0 >= 0; b0 -= NB) {
    const int bn = min(NB, n - b0);
    R s0r = 0, s0i = 0, s1r = 0, s1i = 0;
    if (r < bn) {
      const R* cr = Ar + b0 + r;
      const R* ci = Ai + b0 + r;
      int c = b0 + bn + cg;
      for (; c + 7 * CG < n; c += 8 * CG) {
        R lr[8], li[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          lr[u] = cr[(int64_t)(c + u * CG) * ld];
          li[u] = ci[(int64_t)(c + u * CG) * ld];
        }
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
          s0r += lr[u] * xr[c + u * CG] - li[u] * xi[c + u * CG];
          s0i += lr[u] * xi[c + u * CG] + li[u] * xr[c + u * CG];
          s1r += lr[u + 1] * xr[c + (u + 1) * CG] - li[u + 1] * xi[c + (u + 1) * CG];
          s1i += lr[u + 1] * xi[c + (u + 1) * CG] + li[u + 1] * xr[c + (u + 1) * CG];
        }
      }
      for (; c < n; c += CG) {
        const R l0r = cr[(int64_t)c * ld], l0i = ci[(int64_t)c * ld];
        s0r += l0r * xr[c] - l0i * xi[c];
        s0i += l0r * xi[c] + l0i * xr[c];
      }
    }
    pr_[cg][r] = s0r + s1r;
    pi_[cg][r] = s0i + s1i;
    __syncthreads();
    if (tid < bn) {
      R tr = xr[b0 + tid], ti = xi[b0 + tid];
      for (int q = 0; q < CG; ++q) {
        tr -= pr_[q][tid];
        ti -= pi_[q][tid];
      }
      ar_[tid] = tr;
      ai_[tid] = ti;
    }
    __syncthreads();
    R tr = 0, ti = 0;
    if (r < bn) {
      for (int c = r + cg; c < bn; c += CG) {
        const int64_t o = (int64_t)(b0 + c) * ld + b0 + r;
        const R ur = Ar[o], ui = Ai[o];
        tr += ur * ar_[c] - ui * ai_[c];
        ti += ur * ai_[c] + ui * ar_[c];
      }
    }
    pr_[cg][r] = tr;
    pi_[cg][r] = ti;
    __syncthreads();
    if (tid < bn) {
      R yr = 0, yi = 0;
      for (int q = 0; q < CG; ++q) {
        yr += pr_[q][tid];
        yi += pi_[q][tid];
      }
      xr[b0 + tid] = yr;
      xi[b0 + tid] = yi;
    }
    __syncthreads();
  }
  // prolongation: Boolean partition of unity -> each global unknown is
  // written by its owner only; without weights (OAS) the local results go
  // to a buffer that a gather sums in a fixed order
  if (ys) {
    double2* yc = ys + (int64_t)col * ystride + poff[s];
    for (int i = tid; i < n; i += 256) yc[i] = make_double2((double)xr[i], (double)xi[i]);
  } else {
    double2* zc = z + (int64_t)col * zstride;
    const uint8_t* w = pou + poff[s];
    for (int i = tid; i < n; i += 256)
      if (w[i]) zc[D[i]] = make_double2((double)xr[i], (double)xi[i]);
  }
}

// z[i] = sum over the subdomains containing i of y_s (fixed order)
__global__ void k_gather_all(int64_t ndof, const int64_t* __restrict__ ptr, const int64_t* __restrict__ pos,
                             const double2* __restrict__ ys, int64_t ystride, double2* __restrict__ z,
                             int64_t zstride, const int* __restrict__ active, int by_multiplicity) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndof) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) acc = cadd(acc, ys[(int64_t)col * ystride + pos[q]]);
  if (by_multiplicity) {
    // D_s = 1 / (number of subdomains containing unknown i) in every subdomain
    const double w = 1.0 / (double)(ptr[i + 1] - ptr[i]);
    acc = make_double2(acc.x * w, acc.y * w);
  }
  z[(int64_t)col * zstride + i] = acc;
}

// ---------------------------------------------------------------------------
// SpMV: y = A x (or y = b - A x), G lanes per row
// ---------------------------------------------------------------------------
template <int G>
__global__ void __launch_bounds__(256) k_spmv(int64_t n, const int64_t* __restrict__ rowptr, const int* __restrict__ cols,
                                              const double2* __restrict__ vals, const double2* __restrict__ x,
                                              int64_t xstride, double2* __restrict__ y, int64_t ystride,
                                              const double2* __restrict__ b, int64_t bstride,
                                              const int* __restrict__ active) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x % G;
  if (row >= n) return;
  const double2* xc = x + (int64_t)col * xstride;
  double sr = 0.0, si = 0.0;
  const int64_t r0 = rowptr[row], r1 = rowptr[row + 1];
  // a lane's entries c, c + G, c + 2G, ... summed in that order; four of them
  // are loaded together (indices and values first, then the x gathers) so
  // that a row's loads are in flight at once
  for (int64_t c = r0 + l; c < r1; c += 4 * G) {
    int ci[4];
    double2 a[4], xv[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = c + u * G;
      ok[u] = e < r1;
      ci[u] = ok[u] ? cols[e] : 0;
      a[u] = ok[u] ? vals[e] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) xv[u] = xc[ci[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (ok[u]) {
        sr += a[u].x * xv[u].x - a[u].y * xv[u].y;
        si += a[u].x * xv[u].y + a[u].y * xv[u].x;
      }
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o, G);
    si += __shfl_xor(si, o, G);
  }
  if (l == 0) {
    if (b) {
      const double2 bv = b[(int64_t)col * bstride + row];
      y[(int64_t)col * ystride + row] = make_double2(bv.x - sr, bv.y - si);
    } else {
      y[(int64_t)col * ystride + row] = make_double2(sr, si);
    }
  }
}

// Several columns at once (the products of all right-hand sides fused, Sec. 5):
// a group of G lanes owns a row and CB columns, so every matrix entry and
// column index is read once per CB columns instead of once per column.  Each
// column is summed in the same lane order and shuffle tree as k_spmv.
template <int G, int CB>
__global__ void __launch_bounds__(256) k_spmm(int64_t n, const int64_t* __restrict__ rowptr, const int* __restrict__ cols,
                                              const double2* __restrict__ vals, const double2* __restrict__ x,
                                              int64_t xstride, double2* __restrict__ y, int64_t ystride,
                                              const double2* __restrict__ b, int64_t bstride, int ncol,
                                              const int* __restrict__ active) {
  const int c0 = blockIdx.y * CB;
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int l = threadIdx.x % G;
  if (row >= n) return;
  bool on[CB];
  bool any = false;
#pragma unroll
  for (int q = 0; q < CB; ++q) {
    on[q] = c0 + q < ncol && (!active || active[c0 + q]);
    any |= on[q];
  }
  if (!any) return;
  double sr[CB], si[CB];
#pragma unroll
  for (int q = 0; q < CB; ++q) sr[q] = si[q] = 0.0;
  const int64_t r0 = rowptr[row], r1 = rowptr[row + 1];
  for (int64_t c = r0 + l; c < r1; c += G) {
    const double2 a = vals[c];
    const int64_t j = cols[c];
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      if (!on[q]) continue;
      const double2 xv = x[(int64_t)(c0 + q) * xstride + j];
      sr[q] += a.x * xv.x - a.y * xv.y;
      si[q] += a.x * xv.y + a.y * xv.x;
    }
  }
#pragma unroll
  for (int q = 0; q < CB; ++q) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
      sr[q] += __shfl_xor(sr[q], o, G);
      si[q] += __shfl_xor(si[q], o, G);
    }
  }
  if (l != 0) return;
#pragma unroll
  for (int q = 0; q < CB; ++q) {
    if (!on[q]) continue;
    const int col = c0 + q;
    if (b) {
      const double2 bv = b[(int64_t)col * bstride + row];
      y[(int64_t)col * ystride + row] = make_double2(bv.x - sr[q], bv.y - si[q]);
    } else {
      y[(int64_t)col * ystride + row] = make_double2(sr[q], si[q]);
    }
  }
}

// Block of right-hand sides given interleaved (xi[j * kIlCols + c], column c
// of unknown j): a half-wave of 32 lanes owns a row and one column per lane,
// so every gather of x reads the 512 contiguous bytes of one unknown's
// columns and the matrix is read once for all of them.  Each lane sums its
// column over the row's entries in order (a different summation order from
// k_spmv).  The 32 x 32 result tile of a block goes through LDS so that the
// column-major output is written in 512-byte runs.
//
// The unknowns of one mesh entity share their row pattern (the degree-r
// Nedelec basis places several unknowns on each edge and face), so rows 2g
// and 2g+1 usually have the same columns.  A half-wave takes such a pair
// together: it checks the pattern with one ballot, then gathers each x row
// once for both rows (half the gathers, which bound this kernel), keeping
// each row's own summation order.  Pairs whose patterns differ are summed
// row by row.
constexpr int kIlCols = 32;
constexpr int kIlRows = 32;   // rows per workgroup

__device__ inline void il_accumulate(const double2 a, const double2 xv, double& sr, double& si) {
  sr += a.x * xv.x - a.y * xv.y;
  si += a.x * xv.y + a.y * xv.x;
}

// one row, entries [r0, r1), this lane's column
__device__ inline void il_row(int64_t r0, int64_t r1, const int* __restrict__ cols,
                              const double2* __restrict__ vals, const double2* __restrict__ xi, int lane, double& sr,
                              double& si) {
  for (int64_t e = r0; e < r1; e += 4) {
    int ci[4];
    double2 a[4], xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool ok = e + u < r1;
      ci[u] = ok ? cols[e + u] : 0;
      a[u] = ok ? vals[e + u] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) xv[u] = xi[(int64_t)ci[u] * kIlCols + lane];
#pragma unroll
    for (int u = 0; u < 4; ++u) il_accumulate(a[u], xv[u], sr, si);
  }
}

// two rows with the same columns: entries [a0, a0 + len) and [b0, b0 + len)
constexpr int kPairUnroll = 4;
__device__ inline void il_row_pair(int64_t a0, int64_t b0, int64_t len, const int* __restrict__ cols,
                                   const double2* __restrict__ vals, const double2* __restrict__ xi, int lane,
                                   double& ar, double& ai, double& br, double& bi) {
  for (int64_t e = 0; e < len; e += kPairUnroll) {
    int ci[kPairUnroll];
    double2 a[kPairUnroll], b[kPairUnroll], xv[kPairUnroll];
#pragma unroll
    for (int u = 0; u < kPairUnroll; ++u) {
      const bool ok = e + u < len;
      ci[u] = ok ? cols[a0 + e + u] : 0;
      a[u] = ok ? vals[a0 + e + u] : make_double2(0.0, 0.0);
      b[u] = ok ? vals[b0 + e + u] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kPairUnroll; ++u) xv[u] = xi[(int64_t)ci[u] * kIlCols + lane];
#pragma unroll
    for (int u = 0; u < kPairUnroll; ++u) {
      il_accumulate(a[u], xv[u], ar, ai);
      il_accumulate(b[u], xv[u], br, bi);
    }
  }
}

__global__ void __launch_bounds__(256, 6) k_spmm_il(int64_t n, int p, const int64_t* __restrict__ rowptr,
                                                 const int* __restrict__ cols, const double2* __restrict__ vals,
                                                 const double2* __restrict__ xi, double2* __restrict__ y,
                                                 int64_t ystride, const double2* __restrict__ b, int64_t bstride) {
  __shared__ double2 tile[kIlRows][kIlCols + 1];
  const int lane = threadIdx.x & 31;
  const int sub = threadIdx.x >> 5;   // 8 half-waves
  const int64_t row0 = (int64_t)blockIdx.x * kIlRows;
  for (int k = sub; k < kIlRows / 2; k += 8) {
    const int64_t ra = row0 + 2 * k, rb = ra + 1;
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
    if (ra < n) {
      const int64_t a0 = rowptr[ra], a1 = rowptr[ra + 1];
      const int64_t b1 = rb < n ? rowptr[rb + 1] : a1;
      bool paired = rb < n && b1 - a1 == a1 - a0;
      if (paired) {
        bool same = true;
        for (int64_t e = lane; e < a1 - a0; e += 32) same = same && cols[a0 + e] == cols[a1 + e];
        const unsigned long long miss = __ballot(!same);
        paired = ((miss >> (threadIdx.x & 32)) & 0xffffffffull) == 0;
      }
      if (paired) {
        il_row_pair(a0, a1, a1 - a0, cols, vals, xi, lane, ar, ai, br, bi);
      } else {
        il_row(a0, a1, cols, vals, xi, lane, ar, ai);
        if (rb < n) il_row(a1, b1, cols, vals, xi, lane, br, bi);
      }
    }
    tile[2 * k][lane] = make_double2(ar, ai);
    tile[2 * k + 1][lane] = make_double2(br, bi);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kIlRows * kIlCols; idx += 256) {
    const int c = idx / kIlRows, r = idx % kIlRows;
    const int64_t row = row0 + r;
    if (row >= n || c >= p) continue;
    double2 v = tile[r][c];
    if (b) {
      const double2 bv = b[(int64_t)c * bstride + row];
      v = make_double2(bv.x - v.x, bv.y - v.y);
    }
    y[(int64_t)c * ystride + row] = v;
  }
}

// xi[j * kIlCols + c] = x[c * xstride + j] for c < p, and 0 for p <= c < 32
// (every lane of k_spmm_il reads its column; unused ones must be finite)
__global__ void __launch_bounds__(256) k_to_interleaved(int64_t n, int p, const double2* __restrict__ x,
                                                        int64_t xstride, double2* __restrict__ xi) {
  __shared__ double2 tile[kIlCols][kIlRows + 1];
  const int64_t j0 = (int64_t)blockIdx.x * kIlRows;
  for (int idx = threadIdx.x; idx < kIlCols * kIlRows; idx += 256) {
    const int c = idx / kIlRows, r = idx % kIlRows;   // reads along j for one column
    const int64_t j = j0 + r;
    tile[c][r] = (j < n && c < p) ? x[(int64_t)c * xstride + j] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < kIlCols * kIlRows; idx += 256) {
    const int r = idx / kIlCols, c = idx % kIlCols;   // writes along c for one unknown
    const int64_t j = j0 + r;
    if (j < n) xi[j * kIlCols + c] = tile[c][r];
  }
}

// ---------------------------------------------------------------------------
// Krylov vector kernels.  Column c of the batch uses V + c*vcol, where
// vector i of the basis is at offset i*ndof.
// ---------------------------------------------------------------------------
constexpr int kChunk = 2048;       // elements per block in reductions
constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
  return t;
}

// part[col][blk][i] = sum_{k in blk} conj(V_i[k]) w[k], i = 0..j
__global__ void __launch_bounds__(kRedThreads) k_dots(int64_t ndof, int nvec, const double2* __restrict__ V,
                                                      int64_t vcol, const double2* __restrict__ w, int64_t wcol,
                                                      double2* __restrict__ part, int nblk, int maxv,
                                                      const int* __restrict__ active) {
  __shared__ double sh[8];
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int64_t k0 = (int64_t)blockIdx.x * kChunk;
  double2 wl[kChunk / kRedThreads];
#pragma unroll
  for (int q = 0; q < kChunk / kRedThreads; ++q) {
    const int64_t k = k0 + threadIdx.x + q * kRedThreads;
    wl[q] = k < ndof ? w[(int64_t)col * wcol + k] : make_double2(0.0, 0.0);
  }
  for (int i = 0; i < nvec; ++i) {
    const double2* vi = V + (int64_t)col * vcol + (int64_t)i * ndof;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int q = 0; q < kChunk / kRedThreads; ++q) {
      const int64_t k = k0 + threadIdx.x + q * kRedThreads;
      if (k < ndof) {
        const double2 a = vi[k];
        sr += a.x * wl[q].x + a.y * wl[q].y;
        si += a.x * wl[q].y - a.y * wl[q].x;
      }
    }
    sr = block_sum(sr, sh);
    si = block_sum(si, sh);
    if (threadIdx.x == 0) part[((int64_t)col * nblk + blockIdx.x) * maxv + i] = make_double2(sr, si);
  }
}

// h[col][i] (+)= sum_blk part[col][blk][i]; one block per (i, col), strided
// partial sums then a fixed-shape tree (deterministic)
__global__ void __launch_bounds__(256) k_reduce_dots(int nvec, int nblk, int maxv, const double2* __restrict__ part,
                                                     double2* __restrict__ h, int accumulate,
                                                     const int* __restrict__ active) {
  __shared__ double sh[8];
  const int col = blockIdx.y, i = blockIdx.x;
  if (active && !active[col]) return;
  if (i >= nvec) return;
  double sr = 0.0, si = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    const double2 a = part[((int64_t)col * nblk + b) * maxv + i];
    sr += a.x;
    si += a.y;
  }
  sr = block_sum(sr, sh);
  si = block_sum(si, sh);
  if (threadIdx.x == 0) {
    double2* o = h + (int64_t)col * maxv + i;
    *o = accumulate ? make_double2(o->x + sr, o->y + si) : make_double2(sr, si);
  }
}

// w -= sum_i V_i hpass[i]
__global__ void k_update(int64_t ndof, int nvec, const double2* __restrict__ V, int64_t vcol, double2* __restrict__ w,
                         int64_t wcol, const double2* __restrict__ hpass, int maxv, const int* __restrict__ active) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  __shared__ double2 hs[256];
  for (int i = threadIdx.x; i < nvec; i += blockDim.x) hs[i] = hpass[(int64_t)col * maxv + i];
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ndof) return;
  double2 acc = w[(int64_t)col * wcol + k];
  for (int i = 0; i < nvec; ++i) {
    const double2 a = V[(int64_t)col * vcol + (int64_t)i * ndof + k];
    acc.x -= a.x * hs[i].x - a.y * hs[i].y;
    acc.y -= a.x * hs[i].y + a.y * hs[i].x;
  }
  w[(int64_t)col * wcol + k] = acc;
}

// part[col][blk] = sum |w|^2 over the block
__global__ void __launch_bounds__(kRedThreads) k_norm2(int64_t ndof, const double2* __restrict__ w, int64_t wcol,
                                                       double* __restrict__ part, int nblk,
                                                       const int* __restrict__ active) {
  __shared__ double sh[8];
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int64_t k0 = (int64_t)blockIdx.x * kChunk;
  double s = 0.0;
  for (int q = 0; q < kChunk / kRedThreads; ++q) {
    const int64_t k = k0 + threadIdx.x + q * kRedThreads;
    if (k < ndof) {
      const double2 a = w[(int64_t)col * wcol + k];
      s += a.x * a.x + a.y * a.y;
    }
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[(int64_t)col * nblk + blockIdx.x] = s;
}

__global__ void k_reduce_norm(int nblk, const double* __restrict__ part, double* __restrict__ out,
                              const int* __restrict__ active) {
  const int col = blockIdx.x;
  if (active && !active[col]) return;
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += part[(int64_t)col * nblk + b];
    out[col] = sqrt(a);
  }
}

// y = alpha * x  (alpha = 1 / norm[col])
__global__ void k_scale_inv(int64_t ndof, const double2* __restrict__ x, int64_t xcol, double2* __restrict__ y,
                            int64_t ycol, const double* __restrict__ norm, const int* __restrict__ active) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ndof) return;
  const double nv = norm[col];
  const double a = nv > 0.0 ? 1.0 / nv : 0.0;
  const double2 v = x[(int64_t)col * xcol + k];
  y[(int64_t)col * ycol + k] = make_double2(a * v.x, a * v.y);
}

// Arnoldi step j, one thread per column: H(:,j) = h (sum of both passes),
// H(j+1,j) = ||w||; apply the previous rotations, form the new one, update g.
// est[col] = |g_{j+1}|.
__global__ void k_givens(int ncol, int j, int maxv, const double2* __restrict__ h, const double* __restrict__ hn,
                         double2* __restrict__ H, int ldh, double* __restrict__ cs, double2* __restrict__ sn,
                         double2* __restrict__ g, double* __restrict__ est, const int* __restrict__ active) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  if (active && !active[col]) return;
  double2* Hc = H + (int64_t)col * ldh * maxv;      // column-major (maxv rows)
  double* csc = cs + (int64_t)col * maxv;
  double2* snc = sn + (int64_t)col * maxv;
  double2* gc = g + (int64_t)col * (maxv + 1);
  double2* hj = Hc + (int64_t)j * maxv;
  for (int i = 0; i <= j; ++i) hj[i] = h[(int64_t)col * maxv + i];
  hj[j + 1] = make_double2(hn[col], 0.0);
  for (int i = 0; i < j; ++i) {   // [c s; -conj(s) c]
    const double c = csc[i];
    const double2 s = snc[i];
    const double2 a = hj[i], b = hj[i + 1];
    const double2 t = cadd(make_double2(c * a.x, c * a.y), cmul(s, b));
    const double2 u = csub(make_double2(c * b.x, c * b.y), cmul(make_double2(s.x, -s.y), a));
    hj[i] = t;
    hj[i + 1] = u;
  }
  const double2 a = hj[j], b = hj[j + 1];
  const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
  double c;
  double2 s;
  if (nb == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
  } else if (na == 0.0) {
    c = 0.0;
    s = make_double2(b.x / nb, -b.y / nb);
  } else {
    const double nu = hypot(na, nb);
    c = na / nu;
    const double2 ph = make_double2(a.x / na, a.y / na);
    s = cmul(ph, make_double2(b.x / nu, -b.y / nu));
  }
  csc[j] = c;
  snc[j] = s;
  hj[j] = cadd(make_double2(c * a.x, c * a.y), cmul(s, b));
  hj[j + 1] = make_double2(0.0, 0.0);
  const double2 gj = gc[j];
  gc[j + 1] = cmul(make_double2(-s.x, s.y), gj);   // -conj(s) g_j
  gc[j] = make_double2(c * gj.x, c * gj.y);
  est[col] = hypot(gc[j + 1].x, gc[j + 1].y);
}

// y = R^{-1} g (upper triangular, jd x jd), one thread per column
__global__ void k_backsolve(int ncol, const int* __restrict__ jd, int maxv, const double2* __restrict__ H, int ldh,
                            const double2* __restrict__ g, double2* __restrict__ y) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncol) return;
  const int n = jd[col];
  const double2* Hc = H + (int64_t)col * ldh * maxv;
  const double2* gc = g + (int64_t)col * (maxv + 1);
  double2* yc = y + (int64_t)col * maxv;
  for (int i = n - 1; i >= 0; --i) {
    double2 t = gc[i];
    for (int q = i + 1; q < n; ++q) t = csub(t, cmul(Hc[(int64_t)q * maxv + i], yc[q]));
    const double2 d = Hc[(int64_t)i * maxv + i];
    const double den = d.x * d.x + d.y * d.y;
    yc[i] = make_double2((t.x * d.x + t.y * d.y) / den, (t.y * d.x - t.x * d.y) / den);
  }
}

// x += sum_{i<jd} Z_i y_i
__global__ void k_xupdate(int64_t ndof, const int* __restrict__ jd, const double2* __restrict__ Z, int64_t zcol,
                          const double2* __restrict__ y, int maxv, double2* __restrict__ x, int64_t xcol) {
  const int col = blockIdx.y;
  const int n = jd[col];
  if (n == 0) return;
  __shared__ double2 ys[256];
  for (int i = threadIdx.x; i < n; i += blockDim.x) ys[i] = y[(int64_t)col * maxv + i];
  __syncthreads();
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ndof) return;
  double2 acc = x[(int64_t)col * xcol + k];
  for (int i = 0; i < n; ++i) acc = cadd(acc, cmul(Z[(int64_t)col * zcol + (int64_t)i * ndof + k], ys[i]));
  x[(int64_t)col * xcol + k] = acc;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename R>
void launch_local_solve(hipStream_t st, const LocalSolveArgs& a, const R* F, const double2* v, int64_t vstride,
                        double2* z, int64_t zstride, double2* ys, int64_t ystride, int ncol, const int* active) {
  if (a.n_sub == 0 || ncol == 0) return;
  const size_t dyn = 2 * sizeof(R) * (size_t)a.max_ns;
  timed_launch(k_local_solve<R, kLuNB>, dim3(a.n_sub, ncol), dim3(256), (unsigned)dyn, st, F, a.foff, a.nsz, a.lds,
               a.perm, a.poff, a.sub_dofs, a.pou, v, vstride, z, zstride, ys, ystride, active, a.order);
}
template void launch_local_solve<double>(hipStream_t, const LocalSolveArgs&, const double*, const double2*, int64_t,
                                         double2*, int64_t, double2*, int64_t, int, const int*);
template void launch_local_solve<float>(hipStream_t, const LocalSolveArgs&, const float*, const double2*, int64_t,
                                        double2*, int64_t, double2*, int64_t, int, const int*);

hipError_t prepare_local_solve(size_t dyn_bytes_double, size_t dyn_bytes_float) {
  hipError_t e = hipFuncSetAttribute((const void*)k_local_solve<double, kLuNB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes_double);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_local_solve<float, kLuNB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)dyn_bytes_float);
}

void launch_gather_all(hipStream_t st, int64_t ndof, const int64_t* ptr, const int64_t* pos, const double2* ys,
                       int64_t ystride, double2* z, int64_t zstride, int ncol, const int* active,
                       int by_multiplicity) {
  if (ndof == 0 || ncol == 0) return;
  hipLaunchKernelGGL(k_gather_all, dim3((unsigned)((ndof + 255) / 256), ncol), dim3(256), 0, st, ndof, ptr, pos, ys,
                     ystride, z, zstride, active, by_multiplicity);
}

constexpr int kSpmmCols = 8;   // columns per k_spmm group

template <int G>
static void spmv_g(hipStream_t st, unsigned nb, int64_t n, const int64_t* rowptr, const int* cols,
                   const double2* vals, const double2* x, int64_t xstride, double2* y, int64_t ystride,
                   const double2* b, int64_t bstride, int ncol, const int* active) {
  if (ncol == 1)
    timed_launch(k_spmv<G>, dim3(nb, 1), dim3(256), 0, st, n, rowptr, cols, vals, x, xstride, y, ystride, b, bstride,
                 active);
  else
    timed_launch(k_spmm<G, kSpmmCols>, dim3(nb, (ncol + kSpmmCols - 1) / kSpmmCols), dim3(256), 0, st, n, rowptr,
                 cols, vals, x, xstride, y, ystride, b, bstride, ncol, active);
}

void launch_spmv(hipStream_t st, int group, int64_t n, const int64_t* rowptr, const int* cols, const double2* vals,
                 const double2* x, int64_t xstride, double2* y, int64_t ystride, const double2* b, int64_t bstride,
                 int ncol, const int* active) {
  if (n == 0 || ncol == 0) return;
  const unsigned nb = (unsigned)((n * group + 255) / 256);
  switch (group) {
    case 4: spmv_g<4>(st, nb, n, rowptr, cols, vals, x, xstride, y, ystride, b, bstride, ncol, active); break;
    case 8: spmv_g<8>(st, nb, n, rowptr, cols, vals, x, xstride, y, ystride, b, bstride, ncol, active); break;
    case 16: spmv_g<16>(st, nb, n, rowptr, cols, vals, x, xstride, y, ystride, b, bstride, ncol, active); break;
    default: spmv_g<32>(st, nb, n, rowptr, cols, vals, x, xstride, y, ystride, b, bstride, ncol, active); break;
  }
}

void launch_spmm_interleaved(hipStream_t st, int64_t n, int p, const int64_t* rowptr, const int* cols,
                             const double2* vals, const double2* x, int64_t xstride, double2* xi, double2* y,
                             int64_t ystride, const double2* b, int64_t bstride) {
  if (n == 0 || p == 0) return;
  const unsigned nb = (unsigned)((n + kIlRows - 1) / kIlRows);
  if (x) hipLaunchKernelGGL(k_to_interleaved, dim3(nb), dim3(256), 0, st, n, p, x, xstride, xi);
  timed_launch(k_spmm_il, dim3(nb), dim3(256), 0, st, n, p, rowptr, cols, vals, xi, y, ystride, b, bstride);
}

void launch_to_interleaved(hipStream_t st, int64_t n, int p, const double2* x, int64_t xstride, double2* xi) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_to_interleaved, dim3((unsigned)((n + kIlRows - 1) / kIlRows)), dim3(256), 0, st, n, p, x,
                     xstride, xi);
}

int interleaved_cols() { return kIlCols; }

int red_blocks(int64_t ndof) { return (int)((ndof + kChunk - 1) / kChunk); }

void launch_dots(hipStream_t st, int64_t ndof, int nvec, const double2* V, int64_t vcol, const double2* w,
                 int64_t wcol, double2* part, int maxv, int ncol, const int* active) {
  const int nb = red_blocks(ndof);
  hipLaunchKernelGGL(k_dots, dim3(nb, ncol), dim3(kRedThreads), 0, st, ndof, nvec, V, vcol, w, wcol, part, nb, maxv,
                     active);
}

void launch_reduce_dots(hipStream_t st, int64_t ndof, int nvec, const double2* part, double2* h, int maxv,
                        int accumulate, int ncol, const int* active) {
  hipLaunchKernelGGL(k_reduce_dots, dim3(nvec, ncol), dim3(256), 0, st, nvec, red_blocks(ndof), maxv, part, h,
                     accumulate, active);
}

void launch_update(hipStream_t st, int64_t ndof, int nvec, const double2* V, int64_t vcol, double2* w, int64_t wcol,
                   const double2* hpass, int maxv, int ncol, const int* active) {
  hipLaunchKernelGGL(k_update, dim3((unsigned)((ndof + 255) / 256), ncol), dim3(256), 0, st, ndof, nvec, V, vcol, w,
                     wcol, hpass, maxv, active);
}

void launch_norm(hipStream_t st, int64_t ndof, const double2* w, int64_t wcol, double* part, double* out, int ncol,
                 const int* active) {
  const int nb = red_blocks(ndof);
  hipLaunchKernelGGL(k_norm2, dim3(nb, ncol), dim3(kRedThreads), 0, st, ndof, w, wcol, part, nb, active);
  hipLaunchKernelGGL(k_reduce_norm, dim3(ncol), dim3(64), 0, st, nb, part, out, active);
}

void launch_scale_inv(hipStream_t st, int64_t ndof, const double2* x, int64_t xcol, double2* y, int64_t ycol,
                      const double* norm, int ncol, const int* active) {
  hipLaunchKernelGGL(k_scale_inv, dim3((unsigned)((ndof + 255) / 256), ncol), dim3(256), 0, st, ndof, x, xcol, y, ycol,
                     norm, active);
}

void launch_givens(hipStream_t st, int ncol, int j, int maxv, const double2* h, const double* hn, double2* H, int ldh,
                   double* cs, double2* sn, double2* g, double* est, const int* active) {
  hipLaunchKernelGGL(k_givens, dim3((ncol + 63) / 64), dim3(64), 0, st, ncol, j, maxv, h, hn, H, ldh, cs, sn, g, est,
                     active);
}

void launch_backsolve(hipStream_t st, int ncol, const int* jd, int maxv, const double2* H, int ldh, const double2* g,
                      double2* y) {
  hipLaunchKernelGGL(k_backsolve, dim3((ncol + 63) / 64), dim3(64), 0, st, ncol, jd, maxv, H, ldh, g, y);
}

void launch_xupdate(hipStream_t st, int64_t ndof, const int* jd, const double2* Z, int64_t zcol, const double2* y,
                    int maxv, double2* x, int64_t xcol, int ncol) {
  hipLaunchKernelGGL(k_xupdate, dim3((unsigned)((ndof + 255) / 256), ncol), dim3(256), 0, st, ndof, jd, Z, zcol, y,
                     maxv, x, xcol);
}

}  // namespace mxw
