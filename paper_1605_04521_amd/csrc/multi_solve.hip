// ORAS application to many right-hand sides at once (the pseudo-block scheme
// of Sec. 5: the operations of all right-hand sides fused for arithmetic
// intensity).  One workgroup per (subdomain, chunk of PC columns): every factor
// strip is read once per chunk and multiplied into all PC columns on MFMA,
// instead of once per column.
//
// Per subdomain and chunk, X (n_s x PC complex, split planes, row-major so a
// row of X is contiguous) lives in a global scratch buffer.  Forward sweep over
// 32-row blocks b:  T_b = X_b - L_{b,<b} X_{<b}  (MFMA, K = rows before b),
// X_b = L_bb^{-1} T_b (the diagonal block holds L_bb^{-1}); backward likewise
// with U and U_bb^{-1}.  The K range of each product is split over the four
// waves, whose 32 x 32 partial products are summed in LDS.
#include "device.h"
#include "kernels.h"

namespace mxw {

constexpr int kMultiPC = 32;   // columns per chunk

template <typename R, int NB, int PC>
__global__ void __launch_bounds__(256) k_local_solve_multi(
    const R* __restrict__ F, const int64_t* __restrict__ foff, const int* __restrict__ nsz,
    const int* __restrict__ lds, const int* __restrict__ perm, const int64_t* __restrict__ poff,
    const int* __restrict__ sub_dofs, const uint8_t* __restrict__ pou, const double2* __restrict__ v, int64_t vstride,
    double2* __restrict__ z, int64_t zstride, R* __restrict__ xbuf, int64_t xchunk, int ncol,
    const int* __restrict__ active, const int* __restrict__ order) {
  static_assert(NB == 32 && PC == 32, "tile shape assumes 32 x 32 blocks");
  typedef typename Mfma<R>::acc_t acc_t;
  // Sr/Si[2]: partial products of the waves, then T_b in slot 0
  __shared__ R Sr[2][NB][PC + 1], Si[2][NB][PC + 1];
  __shared__ R Dr[NB][NB + 1], Di[NB][NB + 1];     // diagonal inverse block [row][col]
  const int s = order ? order[blockIdx.x] : blockIdx.x;
  const int chunk = blockIdx.y, c0 = chunk * PC;
  const int n = nsz[s];
  const int64_t ld = lds[s];
  const R* Ar = F + foff[s];
  const R* Ai = Ar + ld * n;
  const int* P = perm + poff[s];
  const int* D = sub_dofs + poff[s];
  R* Xr = xbuf + (int64_t)chunk * xchunk + 2 * poff[s] * PC;
  R* Xi = Xr + (int64_t)n * PC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;

  for (int idx = tid; idx < n * PC; idx += 256) {
    const int i = idx / PC, c = idx % PC, col = c0 + c;
    double2 a = make_double2(0.0, 0.0);
    if (col < ncol) a = v[(int64_t)col * vstride + D[P[i]]];
    Xr[idx] = (R)a.x;
    Xi[idx] = (R)a.y;
  }
  __syncthreads();

  for (int sweep = 0; sweep < 2; ++sweep) {
    const int nblk = (n + NB - 1) / NB;
    for (int bq = 0; bq < nblk; ++bq) {
      const int b = sweep == 0 ? bq : nblk - 1 - bq;
      const int b0 = b * NB, bn = min(NB, n - b0);
      // K range: [0, b0) forward, [b0 + bn, n) backward, split over the
      // waves in 32-wide slices (slice q goes to wave q mod 4); every wave
      // forms the whole 32 x 32 partial product of its slices, so each
      // factor entry and each entry of X is loaded once per workgroup
      const int k_lo = sweep == 0 ? 0 : b0 + bn, k_hi = sweep == 0 ? b0 : n;
      acc_t pre[2][2], pim[2][2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          pre[rt][ct] = acc_t{0, 0, 0, 0};
          pim[rt][ct] = acc_t{0, 0, 0, 0};
        }
      bool row_ok[2];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) row_ok[rt] = rt * 16 + li < bn;
      for (int k0 = k_lo + 32 * wave; k0 < k_hi; k0 += 128) {
        R ar[2][8], ai[2][8], xr[2][8], xi[2][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int kk = k0 + 4 * u + lk;
          const bool ok = kk < k_hi;
#pragma unroll
          for (int rt = 0; rt < 2; ++rt) {
            const int64_t o = (int64_t)kk * ld + b0 + rt * 16 + li;
            ar[rt][u] = (ok && row_ok[rt]) ? Ar[o] : R(0);
            ai[rt][u] = (ok && row_ok[rt]) ? Ai[o] : R(0);
          }
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) {
            const int64_t o = (int64_t)kk * PC + ct * 16 + li;
            xr[ct][u] = ok ? Xr[o] : R(0);
            xi[ct][u] = ok ? Xi[o] : R(0);
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
              pre[rt][ct] = Mfma<R>::op(ar[rt][u], xr[ct][u], pre[rt][ct]);
              pre[rt][ct] = Mfma<R>::op(-ai[rt][u], xi[ct][u], pre[rt][ct]);
              pim[rt][ct] = Mfma<R>::op(ar[rt][u], xi[ct][u], pim[rt][ct]);
              pim[rt][ct] = Mfma<R>::op(ai[rt][u], xr[ct][u], pim[rt][ct]);
            }
      }
      // sum the four partial products: waves 0,1 store, waves 2,3 add
      for (int phase = 0; phase < 2; ++phase) {
        if ((wave >> 1) == phase) {
          const int slot = wave & 1;
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int r = rt * 16 + Mfma<R>::row(lane, q), c = ct * 16 + li;
                if (phase == 0) {
                  Sr[slot][r][c] = pre[rt][ct][q];
                  Si[slot][r][c] = pim[rt][ct][q];
                } else {
                  Sr[slot][r][c] += pre[rt][ct][q];
                  Si[slot][r][c] += pim[rt][ct][q];
                }
              }
        }
        __syncthreads();
      }
      // T_b = X_b - (L or U) X in slot 0; stage the inverse diagonal block
      for (int idx = tid; idx < NB * PC; idx += 256) {
        const int r = idx / PC, c = idx % PC;
        R tr = R(0), ti = R(0);
        if (r < bn) {
          tr = Xr[(int64_t)(b0 + r) * PC + c] - (Sr[0][r][c] + Sr[1][r][c]);
          ti = Xi[(int64_t)(b0 + r) * PC + c] - (Si[0][r][c] + Si[1][r][c]);
        }
        Sr[0][r][c] = tr;
        Si[0][r][c] = ti;
      }
      for (int idx = tid; idx < NB * NB; idx += 256) {
        const int r = idx % NB, c = idx / NB;
        R vr = R(0), vi = R(0);
        if (r < bn && c < bn) {
          vr = Ar[(int64_t)(b0 + c) * ld + b0 + r];
          vi = Ai[(int64_t)(b0 + c) * ld + b0 + r];
        }
        Dr[r][c] = vr;
        Di[r][c] = vi;
      }
      __syncthreads();
      // X_b = L_bb^{-1} T_b (unit lower, strict part stored) or U_bb^{-1} T_b
      for (int idx = tid; idx < NB * PC; idx += 256) {
        const int r = idx / PC, c = idx % PC;
        if (r >= bn) continue;
        R yr, yi;
        if (sweep == 0) {
          yr = Sr[0][r][c];
          yi = Si[0][r][c];
          for (int q = 0; q < r; ++q) {
            yr += Dr[r][q] * Sr[0][q][c] - Di[r][q] * Si[0][q][c];
            yi += Dr[r][q] * Si[0][q][c] + Di[r][q] * Sr[0][q][c];
          }
        } else {
          yr = R(0);
          yi = R(0);
          for (int q = r; q < bn; ++q) {
            yr += Dr[r][q] * Sr[0][q][c] - Di[r][q] * Si[0][q][c];
            yi += Dr[r][q] * Si[0][q][c] + Di[r][q] * Sr[0][q][c];
          }
        }
        Xr[(int64_t)(b0 + r) * PC + c] = yr;
        Xi[(int64_t)(b0 + r) * PC + c] = yi;
      }
      __syncthreads();
    }
  }
  // Boolean prolongation, active columns only
  const uint8_t* w = pou + poff[s];
  for (int idx = tid; idx < n * PC; idx += 256) {
    const int i = idx / PC, c = idx % PC, col = c0 + c;
    if (col >= ncol || !w[i]) continue;
    if (active && !active[col]) continue;
    z[(int64_t)col * zstride + D[i]] = make_double2((double)Xr[idx], (double)Xi[idx]);
  }
}

template <typename R>
void launch_local_solve_multi(hipStream_t st, const LocalSolveArgs& a, const R* F, const double2* v, int64_t vstride,
                              double2* z, int64_t zstride, R* xbuf, int64_t sum_ns, int ncol, const int* active) {
  if (a.n_sub == 0 || ncol == 0) return;
  const int nchunk = (ncol + kMultiPC - 1) / kMultiPC;
  const int64_t xchunk = 2 * sum_ns * kMultiPC;
  timed_launch(k_local_solve_multi<R, kLuNB, kMultiPC>, dim3(a.n_sub, nchunk), dim3(256), 0, st, F, a.foff, a.nsz,
               a.lds, a.perm, a.poff, a.sub_dofs, a.pou, v, vstride, z, zstride, xbuf, xchunk, ncol, active, a.order);
}
template void launch_local_solve_multi<double>(hipStream_t, const LocalSolveArgs&, const double*, const double2*,
                                               int64_t, double2*, int64_t, double*, int64_t, int, const int*);
template void launch_local_solve_multi<float>(hipStream_t, const LocalSolveArgs&, const float*, const double2*,
                                              int64_t, double2*, int64_t, float*, int64_t, int, const int*);

int multi_chunk_cols() { return kMultiPC; }

}  // namespace mxw
