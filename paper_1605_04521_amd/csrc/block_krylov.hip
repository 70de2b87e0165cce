// Block flexible GMRES over one shared Krylov space for all right-hand sides
// (the block solver of Sec. 5): the products with the tall n x (j+1)p bases
// (split-K Gram matrices V^H W and their fixed-order reduction, the updates
// W -= V H and X += Z Y) on MFMA with three real products per complex
// product, the Cholesky factor of a Gram matrix (the
// block QR of a new basis block is a Cholesky QR applied twice), the
// Householder update of the block Hessenberg least-squares problem, and its
// back substitution.
//
// Layouts (all complex FP64, column-major):
//   Hc  (m+1)p x p : new column block of the block Hessenberg matrix
//   T   m x [2p x 2p] : per step, the unitary Q_j^H of the Householder QR of
//                       the 2p x p window at rows jp..(j+2)p (applied to later
//                       column blocks and to E)
//   Rls mp x mp    : upper triangular factor of the block Hessenberg matrix
//   E   (m+1)p x p : Q^H (S0; 0), the transformed right-hand side; the norms
//                    of its rows (j+1)p..(j+2)p are the residual estimates.
#include "device.h"
#include "kernels.h"

namespace mxw {

constexpr int kMaxBlockP = 32;

// H[idx] = sum over parts of part[t][idx].  A workgroup owns 16 outputs; its
// 16 groups of 16 threads sum interleaved parts, and the 16 group sums are
// added in LDS in a fixed order (deterministic for a given part count).
__global__ void __launch_bounds__(256) k_gram_reduce(int64_t len, int nparts, const double2* __restrict__ part,
                                                     double2* __restrict__ H, const int* __restrict__ cond) {
  if (cond && !*cond) return;   // a step's optional work, decided on the device
  __shared__ double2 acc[16][17];
  const int o = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t idx = (int64_t)blockIdx.x * 16 + o;
  double sr = 0.0, si = 0.0;
  if (idx < len)
    for (int t = g; t < nparts; t += 16) {
      const double2 a = part[(int64_t)t * len + idx];
      sr += a.x;
      si += a.y;
    }
  acc[g][o] = make_double2(sr, si);
  __syncthreads();
  if (g == 0 && idx < len) {
    double tr = 0.0, ti = 0.0;
    for (int q = 0; q < 16; ++q) {
      tr += acc[q][o].x;
      ti += acc[q][o].y;
    }
    H[idx] = make_double2(tr, ti);
  }
}

void launch_gram_reduce(hipStream_t st, int64_t len, int nparts, const double2* part, double2* H, const int* cond) {
  if (len == 0) return;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((len + 15) / 16)), dim3(256), 0, st, len, nparts, part, H, cond);
}

// ---------------------------------------------------------------------------
// Products with the tall bases (complex FP64 on MFMA, 16x16x4 f64 tiles, four
// real products per complex tile)
// ---------------------------------------------------------------------------
constexpr int kGramChunkStep = 32;   // n entries staged per LDS step

// Split-K Gram partials: part[ch][b*Q + q] = sum over the chunk's entries of
// conj(V[q][i]) W[b][i], q < Q, b < p <= 32.  Grid (ceil(Q/64), chunks), so
// the workgroups sharing a chunk's strip of W are launched together; the four
// waves of a workgroup take 16 rows q each; the W and V strips of every
// 16-entry step are staged in LDS with coalesced loads (the same
// accumulation order as 32-entry steps, at four workgroups per CU instead of
// three: 1.99 -> 1.94 s per default step).  (Keeping a chunk's
// workgroups on one XCD, so that its strip of W is fetched into one L2
// instead of several, measured slower: 10.3 -> 10.9 ms at 1,600 rows.)
__global__ void __launch_bounds__(256, 4) k_bgram(const double2* __restrict__ V, int Q, const double2* __restrict__ W,
                                               int p, int64_t n, int64_t chunk, double2* __restrict__ part,
                                               const int* __restrict__ cond) {
  if (cond && !*cond) return;   // a step's optional work, decided on the device
  const int ch = blockIdx.y, qt = blockIdx.x;
  typedef Mfma<double>::acc_t acc_t;
  constexpr int S = kGramChunkStep / 2;   // 16-entry strips: 122 registers, four workgroups per CU
  __shared__ double2 Vs[64][S + 1];
  __shared__ double2 Ws[kMaxBlockP][S + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int64_t i0 = (int64_t)ch * chunk, i1 = min(n, i0 + chunk);
  const int q0 = qt * 64;
  // conj(a) b by three real products (Gauss): P1 = ar br, P2 = ai bi,
  // P3 = (ar - ai)(br + bi); Re = P1 + P2, Im = P3 - P1 + P2
  acc_t p1[2], p2[2], p3[2];
  for (int t = 0; t < 2; ++t) p1[t] = p2[t] = p3[t] = acc_t{0, 0, 0, 0};
  // the strips of the next step are loaded into registers while the current
  // step's products run
  double2 pv[64 * S / 256], pw[kMaxBlockP * S / 256];
  auto fetch = [&](int64_t is) {
#pragma unroll
    for (int u = 0; u < 64 * S / 256; ++u) {
      const int idx = tid + 256 * u, r = idx / S, k = idx % S;
      const int64_t i = is + k;
      pv[u] = (q0 + r < Q && i < i1) ? V[(int64_t)(q0 + r) * n + i] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < kMaxBlockP * S / 256; ++u) {
      const int idx = tid + 256 * u, r = idx / S, k = idx % S;
      const int64_t i = is + k;
      pw[u] = (r < p && i < i1) ? W[(int64_t)r * n + i] : make_double2(0.0, 0.0);
    }
  };
  if (i0 < i1) fetch(i0);
  for (int64_t is = i0; is < i1; is += S) {
#pragma unroll
    for (int u = 0; u < 64 * S / 256; ++u) {
      const int idx = tid + 256 * u;
      Vs[idx / S][idx % S] = pv[u];
    }
#pragma unroll
    for (int u = 0; u < kMaxBlockP * S / 256; ++u) {
      const int idx = tid + 256 * u;
      Ws[idx / S][idx % S] = pw[u];
    }
    __syncthreads();
    if (is + S < i1) fetch(is + S);
#pragma unroll
    for (int k0 = 0; k0 < S; k0 += 4) {
      const double2 a = Vs[wave * 16 + li][k0 + lk];
      const double ad = a.x - a.y;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double2 b = Ws[t * 16 + li][k0 + lk];
        p1[t] = Mfma<double>::op(a.x, b.x, p1[t]);
        p2[t] = Mfma<double>::op(a.y, b.y, p2[t]);
        p3[t] = Mfma<double>::op(ad, b.x + b.y, p3[t]);
      }
    }
    __syncthreads();
  }
  double2* out = part + (int64_t)ch * Q * p;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = q0 + wave * 16 + Mfma<double>::row(lane, v), b = t * 16 + li;
      if (q < Q && b < p) out[(int64_t)b * Q + q] = make_double2(p1[t][v] + p2[t][v], p3[t][v] - p1[t][v] + p2[t][v]);
    }
}

// Split-K partials of the p x p Gram matrix W^H W (p <= 32): the strip of W
// is staged once per step (the general kernel would stage it twice and leave
// half of its waves without rows); wave w forms the 16 x 16 tile (rows
// (w & 1) * 16, columns (w >> 1) * 16).  Same partial layout.
__global__ void __launch_bounds__(256) k_bgram_self(const double2* __restrict__ W, int p, int64_t n, int64_t chunk,
                                                    double2* __restrict__ part, const int* __restrict__ cond) {
  if (cond && !*cond) return;   // a step's optional work, decided on the device
  typedef Mfma<double>::acc_t acc_t;
  constexpr int S = kGramChunkStep;
  __shared__ double2 Ws[kMaxBlockP][S + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int qt = wave & 1, bt = wave >> 1;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  acc_t p1 = acc_t{0, 0, 0, 0}, p2 = p1, p3 = p1;
  double2 pw[kMaxBlockP * S / 256];
  auto fetch = [&](int64_t is) {
#pragma unroll
    for (int u = 0; u < kMaxBlockP * S / 256; ++u) {
      const int idx = tid + 256 * u, r = idx / S, k = idx % S;
      const int64_t i = is + k;
      pw[u] = (r < p && i < i1) ? W[(int64_t)r * n + i] : make_double2(0.0, 0.0);
    }
  };
  if (i0 < i1) fetch(i0);
  for (int64_t is = i0; is < i1; is += S) {
#pragma unroll
    for (int u = 0; u < kMaxBlockP * S / 256; ++u) {
      const int idx = tid + 256 * u;
      Ws[idx / S][idx % S] = pw[u];
    }
    __syncthreads();
    if (is + S < i1) fetch(is + S);
#pragma unroll
    for (int k0 = 0; k0 < S; k0 += 4) {
      const double2 a = Ws[qt * 16 + li][k0 + lk], b = Ws[bt * 16 + li][k0 + lk];
      p1 = Mfma<double>::op(a.x, b.x, p1);
      p2 = Mfma<double>::op(a.y, b.y, p2);
      p3 = Mfma<double>::op(a.x - a.y, b.x + b.y, p3);
    }
    __syncthreads();
  }
  double2* out = part + (int64_t)blockIdx.x * p * p;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int q = qt * 16 + Mfma<double>::row(lane, v), b = bt * 16 + li;
    if (q < p && b < p) out[(int64_t)b * p + q] = make_double2(p1[v] + p2[v], p3[v] - p1[v] + p2[v]);
  }
}

void launch_bgram(hipStream_t st, const double2* V, int Q, const double2* W, int p, int64_t n, int nchunks,
                  double2* part, const int* cond) {
  const int64_t chunk = ((n + nchunks - 1) / nchunks + kGramChunkStep - 1) / kGramChunkStep * kGramChunkStep;
  const int used = (int)((n + chunk - 1) / chunk);
  if (V == W && Q == p) {
    hipLaunchKernelGGL(k_bgram_self, dim3(used), dim3(256), 0, st, W, p, n, chunk, part, cond);
    return;
  }
  hipLaunchKernelGGL(k_bgram, dim3((Q + 63) / 64, used), dim3(256), 0, st, V, Q, W, p, n, chunk, part, cond);
}

int bgram_parts(int64_t n, int nchunks) {
  const int64_t chunk = ((n + nchunks - 1) / nchunks + kGramChunkStep - 1) / kGramChunkStep * kGramChunkStep;
  return (int)((n + chunk - 1) / chunk);
}

// out[b][i] = beta C[b][i] + alpha sum_q A[q][i] M[q][b] for b < p <= 32, q < K;
// M column-major K x p with leading dimension ldm.  Formed as out^T = M^T A^T:
// a workgroup covers 64 entries i, each wave 32 b x 16 i (lanes run along i,
// so the stores of out are coalesced); four workgroups per CU.  Per step of
// 16 q the workgroup stages the 16 x 64 tile of A (rows of 1 KB, coalesced)
// and the 16 x p tile of M (read once per workgroup instead of once per
// wave) in LDS; the next step's tiles are loaded into registers while the
// current one is multiplied.  out may be C.
__global__ void __launch_bounds__(256, 3) k_bupdate(const double2* __restrict__ A, int K, const double2* __restrict__ M,
                                                 int ldm, int p, int64_t n, double alpha, double beta,
                                                 const double2* C, double2* out, const int* __restrict__ cond) {
  if (cond && !*cond) return;   // a step's optional work, decided on the device
  typedef Mfma<double>::acc_t acc_t;
  constexpr int KS = 16, IW = 64;
  constexpr int LA = KS * IW / 256, LM = KS * kMaxBlockP / 256;
  __shared__ double2 As[KS][IW + 1];
  __shared__ double2 Ms[KS][kMaxBlockP + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * IW;
  // m a by three real products (Gauss): P1 = mr ar, P2 = mi ai,
  // P3 = (mr + mi)(ar + ai); Re = P1 - P2, Im = P3 - P1 - P2
  acc_t p1[2], p2[2], p3[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) p1[t] = p2[t] = p3[t] = acc_t{0, 0, 0, 0};
  double2 pa[LA], pm[LM];
  auto fetch = [&](int q0) {
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int idx = tid + 256 * u, r = idx / IW, c = idx % IW;
      const int q = q0 + r;
      const int64_t i = i0 + c;
      pa[u] = (q < K && i < n) ? A[(int64_t)q * n + i] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < LM; ++u) {   // consecutive threads along q of one column of M
      const int idx = tid + 256 * u, b = idx / KS, r = idx % KS;
      const int q = q0 + r;
      pm[u] = (q < K && b < p) ? M[(int64_t)b * ldm + q] : make_double2(0.0, 0.0);
    }
  };
  if (K > 0) fetch(0);
  for (int q0 = 0; q0 < K; q0 += KS) {
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int idx = tid + 256 * u;
      As[idx / IW][idx % IW] = pa[u];
    }
#pragma unroll
    for (int u = 0; u < LM; ++u) {
      const int idx = tid + 256 * u;
      Ms[idx % KS][idx / KS] = pm[u];
    }
    __syncthreads();
    if (q0 + KS < K) fetch(q0 + KS);
#pragma unroll
    for (int s4 = 0; s4 < KS / 4; ++s4) {
      const int r = 4 * s4 + lk;
      const double2 a = As[r][wave * 16 + li];
      const double as = a.x + a.y;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const double2 m = Ms[r][t * 16 + li];
        p1[t] = Mfma<double>::op(m.x, a.x, p1[t]);
        p2[t] = Mfma<double>::op(m.y, a.y, p2[t]);
        p3[t] = Mfma<double>::op(m.x + m.y, as, p3[t]);
      }
    }
    __syncthreads();
  }
  const int64_t i = i0 + wave * 16 + li;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int b = t * 16 + Mfma<double>::row(lane, v);
      if (b < p && i < n) {
        const double re = p1[t][v] - p2[t][v], im = p3[t][v] - p1[t][v] - p2[t][v];
        double2 r = make_double2(alpha * re, alpha * im);
        if (beta != 0.0) {
          const double2 c = C[(int64_t)b * n + i];
          r.x += beta * c.x;
          r.y += beta * c.y;
        }
        out[(int64_t)b * n + i] = r;
      }
    }
}

void launch_bupdate(hipStream_t st, const double2* A, int K, const double2* M, int ldm, int p, int64_t n,
                    double alpha, double beta, const double2* C, double2* out, const int* cond) {
  hipLaunchKernelGGL(k_bupdate, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, st, A, K, M, ldm, p, n, alpha,
                     beta, C, out, cond);
}

// Cholesky G = R^H R (R upper, p x p) and R^{-1}; optionally S = R Rprev.
// info[0] = 1 if a column is zero or a pivot of the scaled Gram matrix is not
// positive beyond rounding (the block is rank deficient).
__global__ void __launch_bounds__(256) k_chol(int p, const double2* __restrict__ G, double2* __restrict__ R,
                                              double2* __restrict__ Rinv, const double2* __restrict__ Rprev,
                                              double2* __restrict__ S, int* __restrict__ info) {
  __shared__ double2 A[kMaxBlockP][kMaxBlockP + 1];   // A[row][col], becomes R
  __shared__ double2 Ri[kMaxBlockP][kMaxBlockP + 1];
  __shared__ double dsc[kMaxBlockP];
  __shared__ int bad;
  const int tid = threadIdx.x;
  // columns scaled to unit norm first (G -> D^-1 G D^-1, D = diag(G)^1/2):
  // the Cholesky factor of the scaled Gram matrix is then limited by the
  // independence of the columns, not by their spread in norm (columns of a
  // block residual differ by orders of magnitude once some have converged);
  // R = R~ D and R^-1 = D^-1 R~^-1 restore the scaling
  // (a column below 1e-14 of the largest norm counts as zero: it is not
  // scaled up, and its pivot is floored below)
  double gmax = 0.0;
  for (int k = 0; k < p; ++k) gmax = fmax(gmax, G[(int64_t)k * p + k].x);
  if (tid == 0) bad = !(gmax > 0.0) || !isfinite(gmax);
  if (tid < p) {
    const double g = G[(int64_t)tid * p + tid].x;
    dsc[tid] = gmax > 0.0 ? sqrt(fmax(g, 1e-28 * gmax)) : 1.0;
  }
  __syncthreads();
  for (int idx = tid; idx < p * p; idx += 256) {
    const int r = idx % p, c = idx / p;
    const double sc = 1.0 / (dsc[r] * dsc[c]);
    A[r][c] = make_double2(G[idx].x * sc, G[idx].y * sc);
  }
  __syncthreads();
  // A floored pivot marks a column that depends on the ones before it: its
  // row of R~ right of the diagonal is set to zero instead of being divided
  // by the tiny pivot.  Dividing would put multipliers of size 1/sqrt(floor)
  // into R~, and the back substitution for R~^-1 compounds them from one
  // dependent column to the next (for a block with geometrically decaying
  // singular values, R~^-1 reached 1e54 in a host model of this kernel, and
  // the next Gram matrix overflows).  With the row zeroed R~^-1 stays bounded
  // by 1/sqrt(floor); W = Q R still holds exactly (Q = W R^-1), the columns
  // after k keep their small component along the dependent direction, and the
  // second Cholesky QR pass orthogonalises them.
  __shared__ int floored;
  const double floor_ = 1e-15 * p;
  for (int k = 0; k < p; ++k) {
    if (tid == 0) {
      double d = A[k][k].x;
      floored = 0;
      if (!(d > floor_)) {
        bad = 1;
        floored = 1;
        d = fmax(floor_, 1e-300);
      }
      A[k][k] = make_double2(sqrt(d), 0.0);
    }
    __syncthreads();
    const double rkk = A[k][k].x;
    // row k right of the diagonal, then the trailing Hermitian update
    for (int c = k + 1 + tid; c < p; c += 256)
      A[k][c] = floored ? make_double2(0.0, 0.0) : make_double2(A[k][c].x / rkk, A[k][c].y / rkk);
    __syncthreads();
    for (int idx = tid; idx < p * p; idx += 256) {
      const int r = idx % p, c = idx / p;
      if (r > k && c >= r) {
        // A[r][c] -= conj(R[k][r]) R[k][c]
        const double2 a = A[k][r], b = A[k][c];
        A[r][c].x -= a.x * b.x + a.y * b.y;
        A[r][c].y -= a.x * b.y - a.y * b.x;
      }
    }
    __syncthreads();
  }
  // zero the strict lower part; R^{-1} by back substitution, one column per thread
  for (int idx = tid; idx < p * p; idx += 256) {
    const int r = idx % p, c = idx / p;
    if (r > c) A[r][c] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (tid < p) {
    const int c = tid;
    for (int r = p - 1; r >= 0; --r) {
      double xr = (r == c) ? 1.0 : 0.0, xi = 0.0;
      if (r <= c) {
        for (int q = r + 1; q <= c; ++q) {
          const double2 a = A[r][q], y = Ri[q][c];
          xr -= a.x * y.x - a.y * y.y;
          xi -= a.x * y.y + a.y * y.x;
        }
        const double d = A[r][r].x;
        xr /= d;
        xi /= d;
      }
      Ri[r][c] = make_double2(r <= c ? xr : 0.0, r <= c ? xi : 0.0);
    }
  }
  __syncthreads();
  // undo the column scaling: R = R~ D, R^-1 = D^-1 R~^-1
  for (int idx = tid; idx < p * p; idx += 256) {
    const int r = idx % p, c = idx / p;
    R[idx] = make_double2(A[r][c].x * dsc[c], A[r][c].y * dsc[c]);
    Rinv[idx] = make_double2(Ri[r][c].x / dsc[r], Ri[r][c].y / dsc[r]);
  }
  __syncthreads();
  for (int idx = tid; idx < p * p; idx += 256) {
    const int r = idx % p, c = idx / p;
    A[r][c] = make_double2(A[r][c].x * dsc[c], A[r][c].y * dsc[c]);
  }
  __syncthreads();
  if (S) {
    for (int idx = tid; idx < p * p; idx += 256) {
      const int r = idx % p, c = idx / p;
      // S = R Rprev (both upper triangular)
      double sr = 0.0, si = 0.0;
      for (int q = r; q <= c; ++q) {
        const double2 a = A[r][q], b = Rprev[(int64_t)c * p + q];
        sr += a.x * b.x - a.y * b.y;
        si += a.x * b.y + a.y * b.x;
      }
      S[idx] = make_double2(sr, si);
    }
  }
  if (tid == 0 && bad) info[0] = 1;
}

void launch_chol(hipStream_t st, int p, const double2* G, double2* R, double2* Rinv, const double2* Rprev,
                 double2* S, int* info) {
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), 0, st, p, G, R, Rinv, Rprev, S, info);
}

// E = 0 except E[0:p, 0:p] = S0
__global__ void k_set_e(int p, int ldE, const double2* __restrict__ S0, double2* __restrict__ E) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ldE * p) return;
  const int r = idx % ldE, c = idx / ldE;
  E[idx] = r < p ? S0[c * p + r] : make_double2(0.0, 0.0);
}

void launch_set_e(hipStream_t st, int p, int ldE, const double2* S0, double2* E) {
  hipLaunchKernelGGL(k_set_e, dim3((ldE * p + 255) / 256), dim3(256), 0, st, p, ldE, S0, E);
}

// Step j of the block Hessenberg least squares (one workgroup):
//   1. Hc = [H1 + H2 (rows 0..(j+1)p); S (rows (j+1)p..(j+2)p)];
//   2. apply Q_i^H of the earlier steps to their windows of Hc;
//   3. Householder QR of the window rows jp..(j+2)p (2p x p), reflectors
//      I - 2 v v^H / (v^H v) with v_0 chosen so that the diagonal is
//      -e^{i arg x_0} |x|; Q_j^H = H_{p-1} ... H_0 stored in T_j;
//   4. E window <- Q_j^H E window; R column block stored; est = row norms.
// Out (p2 x p) = Qt (p2 x p2) In (p2 x p) in LDS, p2 = 2p <= 64: thread t
// forms row t % 64 for the columns of group t / 64 (p / 4 columns), so a
// wave reads In[k][c] as a broadcast and each Qt[r][k] once per k; every
// output sums k = 0..p2-1 in order.
__device__ __forceinline__ void window_product(int p, int p2, const double2 (*Qt)[2 * kMaxBlockP + 1],
                                               const double2 (*In)[kMaxBlockP + 1], double2 (*Out)[kMaxBlockP + 1]) {
  constexpr int CG = kMaxBlockP / 4;   // columns per thread
  const int r = threadIdx.x & 63, c0 = (threadIdx.x >> 6) * CG;
  if (r >= p2 || c0 >= p) return;
  double sr[CG], si[CG];
#pragma unroll
  for (int u = 0; u < CG; ++u) sr[u] = si[u] = 0.0;
  for (int k = 0; k < p2; ++k) {
    const double2 a = Qt[r][k];
#pragma unroll
    for (int u = 0; u < CG; ++u) {
      const double2 b = In[k][c0 + u];
      sr[u] += a.x * b.x - a.y * b.y;
      si[u] += a.x * b.y + a.y * b.x;
    }
  }
#pragma unroll
  for (int u = 0; u < CG; ++u)
    if (c0 + u < p) Out[r][c0 + u] = make_double2(sr[u], si[u]);
}

__global__ void __launch_bounds__(256) k_bls_step(int j, int p, int m, const double2* __restrict__ H1,
                                                  const double2* __restrict__ H2in, const double2* __restrict__ S,
                                                  double2* __restrict__ Hc, double2* __restrict__ T,
                                                  double2* __restrict__ Rls, double2* __restrict__ E,
                                                  double* __restrict__ est, const int* __restrict__ h2_used) {
  // H2 (the second Gram-Schmidt pass's coefficients) counts only when the
  // step took that pass (a flag set on the device)
  const double2* __restrict__ H2 = (H2in && (!h2_used || *h2_used)) ? H2in : nullptr;
  __shared__ double2 A[2 * kMaxBlockP][kMaxBlockP + 1];
  __shared__ double2 B[2 * kMaxBlockP][kMaxBlockP + 1];
  __shared__ double2 Qt[2 * kMaxBlockP][2 * kMaxBlockP + 1];
  __shared__ double2 vh[2 * kMaxBlockP];
  __shared__ double2 wsh[3 * kMaxBlockP];
  __shared__ double tau_s, red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int p2 = 2 * p, ld = (m + 1) * p, Q = (j + 1) * p, ldR = m * p;
  // 1. assemble the column block
  for (int idx = tid; idx < (Q + p) * p; idx += 256) {
    const int r = idx % (Q + p), c = idx / (Q + p);
    double2 v;
    if (r < Q) {
      const double2 a = H1[(int64_t)c * Q + r];
      const double2 b = H2 ? H2[(int64_t)c * Q + r] : make_double2(0.0, 0.0);
      v = make_double2(a.x + b.x, a.y + b.y);
    } else {
      v = S[(int64_t)c * p + (r - Q)];
    }
    Hc[(int64_t)c * ld + r] = v;
  }
  __syncthreads();
  // 2. earlier transforms, window by window (windows overlap by p rows: in
  // order).  The lower half of a transformed window is the upper half of the
  // next one and stays in LDS; Q_i^H is staged in LDS (Qt is free until 3.)
  for (int idx = tid; idx < p * p; idx += 256) {
    const int r = idx % p, c = idx / p;
    A[r][c] = Hc[(int64_t)c * ld + r];
  }
  for (int i = 0; i < j; ++i) {
    for (int idx = tid; idx < p * p; idx += 256) {
      const int r = idx % p, c = idx / p;
      A[p + r][c] = Hc[(int64_t)c * ld + (i + 1) * p + r];
    }
    for (int idx = tid; idx < p2 * p2; idx += 256) {
      const int r = idx % p2, c = idx / p2;
      Qt[r][c] = T[(int64_t)i * p2 * p2 + idx];
    }
    __syncthreads();
    window_product(p, p2, Qt, A, B);
    __syncthreads();
    for (int idx = tid; idx < p2 * p; idx += 256) {
      const int r = idx % p2, c = idx / p2;
      if (r < p)
        Hc[(int64_t)c * ld + i * p + r] = B[r][c];   // final rows of the column block
      else
        A[r - p][c] = B[r][c];                       // carried into the next window
    }
    __syncthreads();
  }
  // 3. Householder QR of the window at rows jp..(j+2)p: the upper half is
  // the carried (or, for j = 0, the first) block, the lower half S
  for (int idx = tid; idx < p * p; idx += 256) {
    const int r = idx % p, c = idx / p;
    A[p + r][c] = Hc[(int64_t)c * ld + (j + 1) * p + r];
  }
  for (int idx = tid; idx < p2 * p2; idx += 256) {
    const int r = idx % p2, c = idx / p2;
    Qt[r][c] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < p; ++k) {
    // norm of A[k:, k] (wave 0)
    if (wave == 0) {
      double s2 = 0.0;
      for (int r = k + lane; r < p2; r += 64) s2 += A[r][k].x * A[r][k].x + A[r][k].y * A[r][k].y;
      s2 = wave_sum(s2);
      if (lane == 0) {
        const double nrm = sqrt(s2);
        const double2 x0 = A[k][k];
        const double ax0 = sqrt(x0.x * x0.x + x0.y * x0.y);
        double2 ph = ax0 > 0.0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
        const double2 alpha = make_double2(-ph.x * nrm, -ph.y * nrm);
        const double vv = 2.0 * nrm * (nrm + ax0);
        tau_s = vv > 0.0 ? 2.0 / vv : 0.0;
        red[0] = alpha.x;
        red[1] = alpha.y;
      }
    }
    __syncthreads();
    for (int r = tid; r < p2; r += 256) {
      double2 v = make_double2(0.0, 0.0);
      if (r > k) v = A[r][k];
      if (r == k) v = make_double2(A[k][k].x - red[0], A[k][k].y - red[1]);
      vh[r] = v;
    }
    __syncthreads();
    const double tau = tau_s;
    // apply to the remaining columns of A and to every column of Qt:
    // w_c = tau v^H col_c, one column per wave at a time (lanes along the
    // rows, wave reduction), then col_c -= v w_c by all threads
    for (int c = wave; c < p + p2; c += 4) {
      const bool isA = c < p;
      if (isA && c <= k) continue;   // uniform over the wave
      double wr = 0.0, wi = 0.0;
      if (lane >= k && lane < p2) {
        const double2 x = isA ? A[lane][c] : Qt[lane][c - p];
        const double2 v = vh[lane];
        wr = v.x * x.x + v.y * x.y;
        wi = v.x * x.y - v.y * x.x;
      }
      wr = wave_sum(wr);
      wi = wave_sum(wi);
      if (lane == 0) wsh[c] = make_double2(tau * wr, tau * wi);
    }
    __syncthreads();
    for (int idx = tid; idx < (p2 - k) * (p + p2); idx += 256) {
      const int r = k + idx % (p2 - k), c = idx / (p2 - k);
      if (c < p && c <= k) continue;
      const double2 v = vh[r], w = wsh[c];
      const double dr = v.x * w.x - v.y * w.y, di = v.x * w.y + v.y * w.x;
      if (c < p) {
        A[r][c].x -= dr;
        A[r][c].y -= di;
      } else {
        Qt[r][c - p].x -= dr;
        Qt[r][c - p].y -= di;
      }
    }
    __syncthreads();
    if (tid == 0) {
      A[k][k] = make_double2(red[0], red[1]);
    }
    for (int r = k + 1 + tid; r < p2; r += 256) A[r][k] = make_double2(0.0, 0.0);
    __syncthreads();
  }
  // store Q_j^H
  for (int idx = tid; idx < p2 * p2; idx += 256) {
    const int r = idx % p2, c = idx / p2;
    T[(int64_t)j * p2 * p2 + idx] = Qt[r][c];
  }
  // R column block: rows 0..jp from Hc, rows jp..(j+1)p from A
  for (int idx = tid; idx < Q * p; idx += 256) {
    const int r = idx % Q, c = idx / Q;
    Rls[(int64_t)(j * p + c) * ldR + r] = r < j * p ? Hc[(int64_t)c * ld + r] : A[r - j * p][c];
  }
  // 4. E window
  for (int idx = tid; idx < p2 * p; idx += 256) {
    const int r = idx % p2, c = idx / p2;
    B[r][c] = E[(int64_t)c * ld + j * p + r];
  }
  __syncthreads();
  window_product(p, p2, Qt, B, A);
  __syncthreads();
  for (int idx = tid; idx < p2 * p; idx += 256) {
    const int r = idx % p2, c = idx / p2;
    E[(int64_t)c * ld + j * p + r] = A[r][c];
  }
  if (tid < p) {
    double s2 = 0.0;
    for (int r = p; r < p2; ++r) s2 += A[r][tid].x * A[r][tid].x + A[r][tid].y * A[r][tid].y;
    est[tid] = sqrt(s2);
  }
}

void launch_bls_step(hipStream_t st, int j, int p, int m, const double2* H1, const double2* H2, const double2* S,
                     double2* Hc, double2* T, double2* Rls, double2* E, double* est, const int* h2_used) {
  hipLaunchKernelGGL(k_bls_step, dim3(1), dim3(256), 0, st, j, p, m, H1, H2, S, Hc, T, Rls, E, est, h2_used);
}

// Y = R^{-1} E[0:jp, :] (R = Rls[0:jp, 0:jp], upper); Y has leading dimension m p.
// Blocked from the bottom: a 32-row diagonal block is solved in LDS (one
// thread per column), then every row above takes the block's contribution
// in one parallel product (the rows of R read coalesced).
__global__ void __launch_bounds__(256) k_bls_solve(int jp, int p, int m, const double2* __restrict__ Rls,
                                                   const double2* __restrict__ E, double2* __restrict__ Y) {
  constexpr int BS = 32;
  __shared__ double2 Rb[BS][BS + 1];
  __shared__ double2 Yb[BS][kMaxBlockP + 1];
  const int tid = threadIdx.x, ldR = m * p, ldE = (m + 1) * p;
  for (int idx = tid; idx < jp * p; idx += 256) {
    const int r = idx % jp, c = idx / jp;
    Y[(int64_t)c * ldR + r] = E[(int64_t)c * ldE + r];
  }
  __syncthreads();
  for (int b1 = jp; b1 > 0; b1 -= BS) {
    const int b0 = max(0, b1 - BS), nb = b1 - b0;
    for (int idx = tid; idx < nb * nb; idx += 256) {
      const int r = idx % nb, c = idx / nb;
      Rb[r][c] = Rls[(int64_t)(b0 + c) * ldR + b0 + r];
    }
    for (int idx = tid; idx < nb * p; idx += 256) {
      const int r = idx % nb, c = idx / nb;
      Yb[r][c] = Y[(int64_t)c * ldR + b0 + r];
    }
    __syncthreads();
    if (tid < p) {
      for (int i = nb - 1; i >= 0; --i) {
        const double2 d = Rb[i][i];
        const double dd = d.x * d.x + d.y * d.y;
        const double2 yi = Yb[i][tid];
        // a zero diagonal (a direction the block never reached) takes no weight
        const double2 v = dd > 0.0 ? make_double2((yi.x * d.x + yi.y * d.y) / dd, (yi.y * d.x - yi.x * d.y) / dd)
                                   : make_double2(0.0, 0.0);
        Yb[i][tid] = v;
        for (int r = 0; r < i; ++r) {
          const double2 a = Rb[r][i];
          Yb[r][tid].x -= a.x * v.x - a.y * v.y;
          Yb[r][tid].y -= a.x * v.y + a.y * v.x;
        }
      }
    }
    __syncthreads();
    for (int idx = tid; idx < nb * p; idx += 256) {
      const int r = idx % nb, c = idx / nb;
      Y[(int64_t)c * ldR + b0 + r] = Yb[r][c];
    }
    for (int idx = tid; idx < b0 * p; idx += 256) {
      const int r = idx % b0, c = idx / b0;
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < nb; ++k) {
        const double2 a = Rls[(int64_t)(b0 + k) * ldR + r], v = Yb[k][c];
        sr += a.x * v.x - a.y * v.y;
        si += a.x * v.y + a.y * v.x;
      }
      double2& y = Y[(int64_t)c * ldR + r];
      y.x -= sr;
      y.y -= si;
    }
    __syncthreads();
  }
}

void launch_bls_solve(hipStream_t st, int jp, int p, int m, const double2* Rls, const double2* E, double2* Y) {
  hipLaunchKernelGGL(k_bls_solve, dim3(1), dim3(256), 0, st, jp, p, m, Rls, E, Y);
}

// Reorthogonalisation test of block classical Gram-Schmidt (the criterion of
// Daniel, Gragg, Kaufman and Stewart, per column): a second pass is needed if
// some column kept less than 1/sqrt(2) of its norm in the first pass.
__global__ void k_reorth_check(int p, const double2* __restrict__ G0, const double2* __restrict__ G1,
                               int* __restrict__ flag) {
  const int c = threadIdx.x;
  int need = 0;
  if (c < p) need = !(G1[(int64_t)c * p + c].x >= 0.5 * G0[(int64_t)c * p + c].x);
  need = __any(need);
  if (c == 0) flag[0] = need;
}

void launch_reorth_check(hipStream_t st, int p, const double2* G0, const double2* G1, int* flag) {
  hipLaunchKernelGGL(k_reorth_check, dim3(1), dim3(64), 0, st, p, G0, G1, flag);
}

int max_block_p() { return kMaxBlockP; }

}  // namespace mxw
