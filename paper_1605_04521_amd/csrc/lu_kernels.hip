#include <algorithm>
// Batched dense complex LU with partial pivoting of the subdomain matrices A_s
// (the factorised local solves A_s^{-1} of ORAS, Sec. 4), in FP64 or FP32.
//
// Storage per subdomain: column-major, leading dimension ld, real plane then
// imaginary plane.  One workgroup (4 wavefronts) factorises one matrix, all
// matrices in one launch (largest first).  Left-looking, block columns of
// width NB = 32; for block column J (columns [j0, j0 + 32)):
//   A-C. the factored part is applied to it: for the 32-row blocks K < J the
//      forward substitution X_K = L_KK^{-1} (X_K - L_{K,<K} X_{<K}), for the
//      rows below X_rows -= L_{rows,<j0} X_{<j0} -- the same blocked sweep as
//      the multi-column local solve (64 rows per pass over the factor, the K
//      range split over the waves, 16x16x4 MFMA products, triangular blocks
//      as MFMA tile products); each factor entry left of j0 is read once per
//      block column; the solved rows (U) also go to a row-major scratch X,
//      the operand layout of the later passes;
//   D. panel: unblocked LU of rows [j0, n) with pivot search on |re| + |im|
//      (lowest row on ties), the search for the next column fused into the
//      rank-1 update of the current one;
//   E. the panel's row interchanges are applied to every other column as one
//      net permutation;
//   F. the diagonal block is replaced by [L_JJ^{-1} strict lower | U_JJ^{-1}],
//      which turns the diagonal solves of every later sweep into products.
// perm receives the row permutation: (P A)[i] = A[perm[i]].
#include "device.h"
#include "kernels.h"
#include "sweep.h"

namespace mxw {

constexpr int kPad = 4;
constexpr int kSub = 8;   // columns of a sub-panel (delayed updates of the panel's later columns)

template <typename R, int NB>
struct PanelSmem {
  // inverse workspace: Are/Aim[c][0..NB) the diagonal block (column c),
  // Are/Aim[c][NB..2NB) column c of L11^{-1}; Bre/Bim[c][0..NB) column c of U11^{-1}
  R Are[NB][2 * NB + kPad];
  R Aim[NB][2 * NB + kPad];
  R Bre[NB][NB + kPad];
  R Bim[NB][NB + kPad];
  double rv[4];
  int ri[4];
  R ur[NB], ui[NB];
  int piv[NB];
  int src[2 * NB], dst[2 * NB];
  int rows[2 * NB], cont[2 * NB];
  int npairs;
};

template <typename R, int NB>
struct SweepSmem {
  R Tr[2 * NB][NB + 1], Ti[2 * NB][NB + 1];        // T of the 64-row pass, overwritten by its solution
  R Br[2][NB][NB + 1], Bi[2][NB][NB + 1];          // [0] first, then second diagonal inverse; [1] coupling block
};

template <typename R, int NB>
union LuSmem {
  PanelSmem<R, NB> p;
  SweepSmem<R, NB> s;
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

// Steps A-C for block column j0 (width kb): 64-row passes over the factored
// columns.  A pass reads its 64 x kb block of the column from the factor
// storage (column-major, coalesced through LDS), subtracts the product with the
// factored part, applies the triangular blocks where the rows are left of j0,
// and writes the result back to the factor storage and, for rows left of j0
// (the only rows later passes use as operand), to the row-major scratch X.
template <typename R, int NB, int KU>
__device__ void update_block_column(SweepSmem<R, NB>& sm, int n, int ld, int j0, int kb, R* __restrict__ Ar,
                                    R* __restrict__ Ai, __amdgpu_buffer_rsrc_t fr, __amdgpu_buffer_rsrc_t fi,
                                    R* __restrict__ Xr, R* __restrict__ Xi, __amdgpu_buffer_rsrc_t xrr,
                                    __amdgpu_buffer_rsrc_t xir) {
  constexpr int PC = NB, SB = 2 * NB;
  typedef typename Mfma<R>::acc_t acc_t;
  const int wave = threadIdx.x >> 6;
  const int rh = wave & 1, kh = wave >> 1;
  const int nsb = (n + SB - 1) / SB;
  for (int sb = 0; sb < nsb; ++sb) {
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, li = lane & 15, lk = lane >> 4;
    const int r0 = sb * SB, rn = min(SB, n - r0);
    const int k_hi = min(r0, j0);                 // product over factored columns [0, k_hi)
    const bool solve0 = r0 < j0, solve1 = r0 + NB < j0;   // blocks left of j0 take the triangular solve
    if (k_hi == 0 && !solve0) continue;           // nothing factored applies to these rows
    const int n0 = min(NB, rn), n1 = max(0, rn - NB);
    // prefetch the triangular blocks (first diagonal, coupling, second diagonal)
    R pbr[3][4], pbi[3][4];
    if (solve0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int idx = tid + 256 * j, r = idx % NB, c = idx / NB;
        const int rows[3] = {0, 1, 1}, cols[3] = {0, 0, 1};
        const int rlim[3] = {n0, n1, n1}, clim[3] = {n0, n0, n1};
        const bool use[3] = {true, true, solve1};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const bool in = use[m] && r < rlim[m] && c < clim[m];
          const int o = in ? ((r0 + cols[m] * NB + c) * ld + r0 + rows[m] * NB + r) * (int)sizeof(R) : kOob;
          pbr[m][j] = BufLoad<R>::at(fr, o);
          pbi[m][j] = BufLoad<R>::at(fi, o);
        }
      }
    }
    // FP32: three real products per complex product (Slice::product3); FP64
    // keeps four (the third accumulator set would spill): p1, p2 = Re, Im
    constexpr bool k3 = sizeof(R) == 4;
    acc_t p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) p1[rt][ct] = p2[rt][ct] = p3[rt][ct] = acc_t{0, 0, 0, 0};
    bool row_ok[2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) row_ok[rt] = rh * NB + rt * 16 + li < rn;
    const int arow = r0 + rh * NB + li;
    for (int k0 = 4 * KU * kh; k0 < k_hi; k0 += 8 * KU) {
      Slice<R, KU, PC> sl;
      sl.load(fr, fi, xrr, xir, ld, arow, row_ok, k0, k_hi, lk, li);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (k3)
        sl.product3(p1, p2, p3);
      else
        sl.product(p1, p2);
    }
    // T = the block of the column (rows r0.., columns j0..j0+kb) - product
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int idx = tid + 256 * j, r = idx % SB, c = idx / SB;
      const int o = (r < rn && c < kb) ? ((j0 + c) * ld + r0 + r) * (int)sizeof(R) : kOob;
      sm.Tr[r][c] = BufLoad<R>::at(fr, o);
      sm.Ti[r][c] = BufLoad<R>::at(fi, o);
    }
    if (solve0) {
      // the diagonal inverses as full matrices (unit lower), identity where
      // the block is right of j0; the coupling block
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int idx = tid + 256 * j, r = idx % NB, c = idx / NB;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          R vr = pbr[m][j], vi = pbi[m][j];
          if (m != 1) {
            const int bn = m == 0 ? n0 : n1;
            vr = c < r ? vr : (c == r && r < bn ? R(1) : R(0));
            vi = c < r ? vi : R(0);
          }
          if (m < 2) {
            sm.Br[m][r][c] = vr;
            sm.Bi[m][r][c] = vi;
          } else {   // kept in registers until the first block is solved
            pbr[2][j] = vr;
            pbi[2][j] = vi;
          }
        }
      }
    }
    __syncthreads();
    for (int phase = 1; phase >= 0; --phase) {
      if (kh == phase) {
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int r = rh * NB + rt * 16 + Mfma<R>::row(lane, q), c = ct * 16 + li;
              if constexpr (k3) {
                sm.Tr[r][c] -= p1[rt][ct][q] - p2[rt][ct][q];
                sm.Ti[r][c] -= p3[rt][ct][q] - p1[rt][ct][q] - p2[rt][ct][q];
              } else {
                sm.Tr[r][c] -= p1[rt][ct][q];
                sm.Ti[r][c] -= p2[rt][ct][q];
              }
            }
      }
      __syncthreads();
    }
    if (solve0) {
      // Y0 = M0 T0 -> rows 0.. of T; T1 -= C Y0; Y1 = M1 T1 -> rows NB.. of T
      const int orow = (wave & 1) * 16, ocol = (wave >> 1) * 16 + li;
      {
        acc_t yre = acc_t{0, 0, 0, 0}, yim = acc_t{0, 0, 0, 0};
        tile_product<R, NB, PC>(sm.Br[0], sm.Bi[0], sm.Tr, sm.Ti, lane, wave, yre, yim);
        __syncthreads();   // every wave has read T0 and M0 before they are overwritten
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = orow + Mfma<R>::row(lane, q);
          sm.Tr[r][ocol] = yre[q];
          sm.Ti[r][ocol] = yim[q];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {   // the second diagonal inverse takes M0's place
          const int idx = tid + 256 * j, r = idx % NB, c = idx / NB;
          sm.Br[0][r][c] = pbr[2][j];
          sm.Bi[0][r][c] = pbi[2][j];
        }
      }
      __syncthreads();
      if (n1 > 0) {
        acc_t cre = acc_t{0, 0, 0, 0}, cim = acc_t{0, 0, 0, 0};
        tile_product<R, NB, PC>(sm.Br[1], sm.Bi[1], sm.Tr, sm.Ti, lane, wave, cre, cim);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = orow + Mfma<R>::row(lane, q);
          sm.Tr[NB + r][ocol] -= cre[q];
          sm.Ti[NB + r][ocol] -= cim[q];
        }
        __syncthreads();
        acc_t yre = acc_t{0, 0, 0, 0}, yim = acc_t{0, 0, 0, 0};
        tile_product<R, NB, PC>(sm.Br[0], sm.Bi[0], sm.Tr + NB, sm.Ti + NB, lane, wave, yre, yim);
        __syncthreads();   // every wave has read T1 before it is overwritten by Y1
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = orow + Mfma<R>::row(lane, q);
          sm.Tr[NB + r][ocol] = yre[q];
          sm.Ti[NB + r][ocol] = yim[q];
        }
      }
      __syncthreads();
      // rows left of j0 to the row-major scratch (operand of later passes)
      const int rsolved = min(rn, j0 - r0);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int idx = tid + 256 * j, r = idx / PC, c = idx % PC;
        if (r < rsolved) {
          Xr[(int64_t)(r0 + r) * PC + c] = sm.Tr[r][c];
          Xi[(int64_t)(r0 + r) * PC + c] = sm.Ti[r][c];
        }
      }
    }
    // the pass's rows back to the factor storage (column-major, coalesced)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int idx = tid + 256 * j, r = idx % SB, c = idx / SB;
      if (r < rn && c < kb) {
        Ar[(int64_t)(j0 + c) * ld + r0 + r] = sm.Tr[r][c];
        Ai[(int64_t)(j0 + c) * ld + r0 + r] = sm.Ti[r][c];
      }
    }
    __syncthreads();
  }
}

// The factorisation of subdomain s by one workgroup (the body of both
// launches below).
template <typename R, int NB, int KU>
__device__ __forceinline__ void lu_subdomain(int s, LuSmem<R, NB>& smu, R* __restrict__ F,
                                             const int64_t* __restrict__ foff, const int* __restrict__ nsz,
                                             const int* __restrict__ lds, int* __restrict__ perm,
                                             const int64_t* __restrict__ poff, R* __restrict__ xscr,
                                             int* __restrict__ info) {
  static_assert(NB == 32, "the sweep tiles assume 32-wide blocks");
  // panel columns updated together per row (fewer in FP64, whose registers
  // are twice as wide)
  constexpr int HC = sizeof(R) == 8 ? 8 : 16;
  PanelSmem<R, NB>& sm = smu.p;
  const int n = nsz[s];
  const int64_t ld = lds[s];
  R* Ar = F + foff[s];
  R* Ai = Ar + ld * n;
  int* P = perm + poff[s];
  R* Xr = xscr + 2 * poff[s] * NB;   // row-major n x NB block column
  R* Xi = Xr + (int64_t)n * NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const __amdgpu_buffer_rsrc_t fr = plane_rsrc(Ar, ld * n * (int64_t)sizeof(R));
  const __amdgpu_buffer_rsrc_t fi = plane_rsrc(Ai, ld * n * (int64_t)sizeof(R));
  const __amdgpu_buffer_rsrc_t xrr = plane_rsrc(Xr, (int64_t)n * NB * sizeof(R));
  const __amdgpu_buffer_rsrc_t xir = plane_rsrc(Xi, (int64_t)n * NB * sizeof(R));
  for (int i = tid; i < n; i += 256) P[i] = i;
  int first_zero = 0;
  // singularity threshold: |pivot| <= n u max|A_s| (FP64) or u max|A_s| (FP32)
  double tiny;
  {
    double amax = 0.0;
    const int nn = n * n;
    for (int e0 = tid; e0 < nn; e0 += 8 * 256) {
      R vr[8], vi[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {   // 8 loads in flight per thread
        const int e = e0 + u * 256;
        const int o = e < nn ? ((e / n) * (int)ld + e % n) * (int)sizeof(R) : kOob;
        vr[u] = BufLoad<R>::at(fr, o);
        vi[u] = BufLoad<R>::at(fi, o);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) amax = fmax(amax, fabs((double)vr[u]) + fabs((double)vi[u]));
    }
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
    // ---- A-C. bring the block column up to date with the factored part
    if (k > 0) update_block_column<R, NB, KU>(smu.s, n, (int)ld, k, kb, Ar, Ai, fr, fi, Xr, Xi, xrr, xir);
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
      // FP32: sub-panel [s0, s_end) of kSub columns: its own columns are
      // updated at every step, the panel's columns right of it once, when it
      // is done.  FP64 updates the whole panel at every step (the delayed
      // update's registers would spill)
      constexpr int kS = sizeof(R) == 4 ? kSub : NB;
      const int s0 = jj / kS * kS, s_end = min(s0 + kS, kb);
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
      // swap rows j and p of the panel; the pivot row goes to LDS
      if (tid < kb) {
        const int64_t c = (int64_t)(k + tid) * ld;
        const R a0 = Ar[c + j], a1 = Ai[c + j], b0 = Ar[c + p], b1 = Ai[c + p];
        if (p != j) {
          Ar[c + j] = b0;
          Ai[c + j] = b1;
          Ar[c + p] = a0;
          Ai[c + p] = a1;
        }
        sm.ur[tid] = b0;
        sm.ui[tid] = b1;
      }
      if (tid == 0) sm.piv[jj] = p;
      __syncthreads();
      const R pr = sm.ur[jj], pi = sm.ui[jj];
      const R den = pr * pr + pi * pi;
      const R rr = den > R(0) ? pr / den : R(0), ri = den > R(0) ? -pi / den : R(0);
      best = -1.0;
      bi = 0x7fffffff;
      // scale column j and update the sub-panel's columns right of it, one
      // row per thread at a time: the row's entries of 16 columns are loaded
      // together (branch-free buffer accesses, masked columns out of range),
      // updated in registers and stored
      for (int i = j + 1 + tid; i < n; i += 512) {
        int row[2] = {i, i + 256};
        int oj[2];
        R lr[2], lim[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          oj[t] = row[t] < n ? (j * (int)ld + row[t]) * (int)sizeof(R) : kOob;
          const R ar = BufLoad<R>::at(fr, oj[t]), ai = BufLoad<R>::at(fi, oj[t]);
          lr[t] = ar * rr - ai * ri;
          lim[t] = ar * ri + ai * rr;
          BufStore<R>::at(fr, oj[t], lr[t]);
          BufStore<R>::at(fi, oj[t], lim[t]);
        }
#pragma nounroll
        for (int h = 0; h < NB; h += HC) {
          if (h + HC <= jj + 1 || h >= s_end) continue;   // uniform: no live column in this part
          R xr[2][HC], xi[2][HC];
          int off[2][HC];
#pragma unroll
          for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < HC; ++u) {
              const int c = h + u;
              off[t][u] = (c > jj && c < s_end && row[t] < n) ? ((k + c) * (int)ld + row[t]) * (int)sizeof(R) : kOob;
              xr[t][u] = BufLoad<R>::at(fr, off[t][u]);
              xi[t][u] = BufLoad<R>::at(fi, off[t][u]);
            }
#pragma unroll
          for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < HC; ++u) {
              const R pr_ = sm.ur[h + u], pi_ = sm.ui[h + u];
              xr[t][u] -= lr[t] * pr_ - lim[t] * pi_;
              xi[t][u] -= lr[t] * pi_ + lim[t] * pr_;
              if (h + u == jj + 1 && row[t] < n) {
                const double v = fabs((double)xr[t][u]) + fabs((double)xi[t][u]);
                if (v > best || (v == best && row[t] < bi)) {
                  best = v;
                  bi = row[t];
                }
              }
              BufStore<R>::at(fr, off[t][u], xr[t][u]);
              BufStore<R>::at(fi, off[t][u], xi[t][u]);
            }
        }
      }
      if (sizeof(R) == 4 && jj + 1 == s_end && s_end < kb) {
        // the sub-panel is factorised: U12 = L11^{-1} A12 on its pivot rows
        // (one thread per later column), then A22 -= L21 U12 on the rows
        // below it, which also yields the next column's pivot candidates
        const int ns = s_end - s0, nc = kb - s_end;
        __syncthreads();
        if (tid < nc) {
          const int c = s_end + tid;
          R ur[kSub], ui[kSub];
#pragma unroll
          for (int i = 0; i < kSub; ++i) {
            if (i >= ns) break;
            const int64_t o = (int64_t)(k + c) * ld + k + s0 + i;
            R xr = Ar[o], xi = Ai[o];
#pragma unroll
            for (int m = 0; m < kSub; ++m) {
              if (m >= i) break;
              const int64_t ol = (int64_t)(k + s0 + m) * ld + k + s0 + i;   // L[s0 + i][s0 + m]
              const R lr = Ar[ol], li = Ai[ol];
              xr -= lr * ur[m] - li * ui[m];
              xi -= lr * ui[m] + li * ur[m];
            }
            ur[i] = xr;
            ui[i] = xi;
            Ar[o] = xr;
            Ai[o] = xi;
            sm.Bre[i][c] = xr;
            sm.Bim[i][c] = xi;
          }
        }
        __syncthreads();
        for (int r = k + s_end + tid; r < n; r += 256) {
          R lr[kSub], li[kSub];
#pragma unroll
          for (int m = 0; m < kSub; ++m) {
            const int o = m < ns ? ((k + s0 + m) * (int)ld + r) * (int)sizeof(R) : kOob;
            lr[m] = BufLoad<R>::at(fr, o);
            li[m] = BufLoad<R>::at(fi, o);
          }
#pragma nounroll
          for (int c0 = s_end; c0 < kb; c0 += 4) {
            R xr[4], xi[4];
            int off[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int c = c0 + u;
              off[u] = c < kb ? ((k + c) * (int)ld + r) * (int)sizeof(R) : kOob;
              xr[u] = BufLoad<R>::at(fr, off[u]);
              xi[u] = BufLoad<R>::at(fi, off[u]);
            }
#pragma unroll
            for (int m = 0; m < kSub; ++m)
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int c = c0 + u;
                const R ur = (m < ns && c < kb) ? sm.Bre[m][c] : R(0), ui = (m < ns && c < kb) ? sm.Bim[m][c] : R(0);
                xr[u] -= lr[m] * ur - li[m] * ui;
                xi[u] -= lr[m] * ui + li[m] * ur;
              }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (c0 + u == s_end) {
                const double v = fabs((double)xr[u]) + fabs((double)xi[u]);
                if (v > best || (v == best && r < bi)) {
                  best = v;
                  bi = r;
                }
              }
              BufStore<R>::at(fr, off[u], xr[u]);
              BufStore<R>::at(fi, off[u], xi[u]);
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
        // 16 columns per wave in flight; masked lanes and the panel's own
        // columns read and write out of range (no-ops)
        for (int c0 = wave * 16; c0 < n; c0 += 64) {
          R vr[16], vi[16];
          int od[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int c = c0 + u;
            const bool ok = lane < np && c < n && (c < k || c >= k + kb);
            const int os = ok ? (c * (int)ld + sr) * (int)sizeof(R) : kOob;
            od[u] = ok ? (c * (int)ld + ds) * (int)sizeof(R) : kOob;
            vr[u] = BufLoad<R>::at(fr, os);
            vi[u] = BufLoad<R>::at(fi, os);
          }
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            BufStore<R>::at(fr, od[u], vr[u]);
            BufStore<R>::at(fi, od[u], vi[u]);
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
    }
    __syncthreads();
  }
  if (tid == 0) info[s] = first_zero;
}

// One workgroup per subdomain (order[blockIdx.x], largest first).
template <typename R, int NB, int KU>
__global__ void __launch_bounds__(256, 2) k_lu(R* __restrict__ F, const int64_t* __restrict__ foff,
                                            const int* __restrict__ nsz, const int* __restrict__ lds,
                                            int* __restrict__ perm, const int64_t* __restrict__ poff,
                                            R* __restrict__ xscr, int* __restrict__ info,
                                            const int* __restrict__ order) {
  __shared__ LuSmem<R, NB> smu;
  lu_subdomain<R, NB, KU>(order ? order[blockIdx.x] : blockIdx.x, smu, F, foff, nsz, lds, perm, poff, xscr, info);
}

// Persistent launch: a grid sized to the resident workgroups takes the
// subdomains from a queue (order[0..count), largest first) until it is
// empty; next is a counter that starts at 0.  Every workgroup leaves once it
// draws an index >= count.
template <typename R, int NB, int KU>
__global__ void __launch_bounds__(256, 2) k_lu_queue(R* __restrict__ F, const int64_t* __restrict__ foff,
                                                  const int* __restrict__ nsz, const int* __restrict__ lds,
                                                  int* __restrict__ perm, const int64_t* __restrict__ poff,
                                                  R* __restrict__ xscr, int* __restrict__ info,
                                                  const int* __restrict__ order, int count, int* __restrict__ next) {
  __shared__ LuSmem<R, NB> smu;
  __shared__ int item;
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd(next, 1);
    __syncthreads();
    const int q = item;
    __syncthreads();   // read by all before thread 0 draws again
    if (q >= count) break;
    lu_subdomain<R, NB, KU>(order ? order[q] : q, smu, F, foff, nsz, lds, perm, poff, xscr, info);
    __syncthreads();
  }
}

__global__ void k_zero_counter(int* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

// ku: k slice width of the block-column update (4 or 8); FP64 always takes 4
// (8 would spill at two workgroups per CU)
template <typename R>
void launch_lu(hipStream_t st, int n_sub, R* F, const int64_t* foff, const int* nsz, const int* lds, int* perm,
               const int64_t* poff, R* scratch, int* info, const int* order, int ku, int* queue) {
  if (n_sub <= 0) return;
  const bool k4 = sizeof(R) == 8 || ku == 4;
  if (queue) {
    // two workgroups per CU stay resident (launch bounds); never more than
    // there are subdomains
    static int cus = 0;
    if (!cus) {
      int dev = 0;
      hipGetDevice(&dev);
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    }
    const int grid = std::min(n_sub, 2 * cus);
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, st, queue);
    if (k4)
      timed_launch(k_lu_queue<R, kLuNB, 4>, dim3(grid), dim3(256), 0, st, F, foff, nsz, lds, perm, poff, scratch,
                   info, order, n_sub, queue);
    else
      timed_launch(k_lu_queue<R, kLuNB, 8>, dim3(grid), dim3(256), 0, st, F, foff, nsz, lds, perm, poff, scratch,
                   info, order, n_sub, queue);
    return;
  }
  if (k4)
    timed_launch(k_lu<R, kLuNB, 4>, dim3(n_sub), dim3(256), 0, st, F, foff, nsz, lds, perm, poff, scratch, info,
                 order);
  else
    timed_launch(k_lu<R, kLuNB, 8>, dim3(n_sub), dim3(256), 0, st, F, foff, nsz, lds, perm, poff, scratch, info,
                 order);
}
template void launch_lu<double>(hipStream_t, int, double*, const int64_t*, const int*, const int*, int*,
                                const int64_t*, double*, int*, const int*, int, int*);
template void launch_lu<float>(hipStream_t, int, float*, const int64_t*, const int*, const int*, int*,
                               const int64_t*, float*, int*, const int*, int, int*);

}  // namespace mxw
