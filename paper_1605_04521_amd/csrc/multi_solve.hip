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
// with U and U_bb^{-1}.  Rows are taken 64 at a time (two diagonal blocks) so
// that X is re-read once per 64 rows; the waves split the 64 rows in halves
// and the K range in two, and the two partial products are summed in LDS.
#include "device.h"
#include "kernels.h"
#include "sweep.h"

namespace mxw {

constexpr int kMultiPC = 32;   // columns per chunk

template <typename R, int NB, int PC, int KU>
__global__ void __launch_bounds__(256) k_local_solve_multi(
    const R* __restrict__ F, const int64_t* __restrict__ foff, const int* __restrict__ nsz,
    const int* __restrict__ lds, const int* __restrict__ perm, const int64_t* __restrict__ poff,
    const int* __restrict__ sub_dofs, const uint8_t* __restrict__ pou, const double2* __restrict__ v, int64_t vstride,
    const double2* __restrict__ vil, double2* __restrict__ z, int64_t zstride, R* __restrict__ xbuf, int64_t xchunk,
    int ncol, const int* __restrict__ active, const int* __restrict__ order) {
  static_assert(NB == 32 && PC == 32, "tile shape assumes 32 x 32 blocks");
  constexpr int SB = 2 * NB;   // rows per pass over the factor
  typedef typename Mfma<R>::acc_t acc_t;
  __shared__ R Tr[SB][PC + 1], Ti[SB][PC + 1];       // T of the super-block
  __shared__ R Br[3][NB][NB + 1], Bi[3][NB][NB + 1];  // diagonal block solved first, coupling block, second diagonal block
  __shared__ R Yr[NB][PC + 1], Yi[NB][PC + 1];       // solution of the block solved first
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
  const int rh = wave & 1, kh = wave >> 1;   // row half of the super-block, half of the K slices
  const __amdgpu_buffer_rsrc_t fr = plane_rsrc(Ar, ld * n * (int64_t)sizeof(R));
  const __amdgpu_buffer_rsrc_t fi = plane_rsrc(Ai, ld * n * (int64_t)sizeof(R));
  const __amdgpu_buffer_rsrc_t xrr = plane_rsrc(Xr, (int64_t)n * PC * sizeof(R));
  const __amdgpu_buffer_rsrc_t xir = plane_rsrc(Xi, (int64_t)n * PC * sizeof(R));

  // restrict and permute: X = P_s R_s v (4 entries in flight per thread)
  for (int base = tid; base < n * PC; base += 4 * 256) {
    double2 a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = base + u * 256;
      a[u] = make_double2(0.0, 0.0);
      if (idx < n * PC) {
        const int i = idx / PC, col = c0 + idx % PC;
        if (col < ncol)   // the interleaved copy: a row's columns in one contiguous read
          a[u] = vil ? vil[(int64_t)D[P[i]] * PC + idx % PC] : v[(int64_t)col * vstride + D[P[i]]];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = base + u * 256;
      if (idx < n * PC) {
        Xr[idx] = (R)a[u].x;
        Xi[idx] = (R)a[u].y;
      }
    }
  }
  __syncthreads();

  const int nsb = (n + SB - 1) / SB;
  for (int sweep = 0; sweep < 2; ++sweep) {
    for (int sq = 0; sq < nsb; ++sq) {
      // lane-derived indices recomputed per pass (an opaque copy of the
      // thread id) instead of being held in registers across the whole kernel
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      const int lane = tid & 63, li = lane & 15, lk = lane >> 4;
      const int sb = sweep == 0 ? sq : nsb - 1 - sq;
      const int r0 = sb * SB, rn = min(SB, n - r0);
      // 32-row blocks in solve order: forward 0 then 1, backward 1 then 0
      const int bf = sweep == 0 ? 0 : 1, bs = 1 - bf;
      const int nf = max(0, min(NB, rn - bf * NB)), ns = max(0, min(NB, rn - bs * NB));
      // prefetch, before the long product: the three factor blocks of the
      // triangular part
      R pbr[3][4], pbi[3][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int idx = tid + 256 * j, r = idx % NB, c = idx / NB;
        const int rows[3] = {bf, bs, bs}, cols[3] = {bf, bf, bs};
        const int rlim[3] = {nf, ns, ns}, clim[3] = {nf, nf, ns};
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const bool in = r < rlim[m] && c < clim[m];
          const int o = in ? ((r0 + cols[m] * NB + c) * (int)ld + r0 + rows[m] * NB + r) * (int)sizeof(R) : kOob;
          pbr[m][j] = BufLoad<R>::at(fr, o);
          pbi[m][j] = BufLoad<R>::at(fi, o);
        }
      }
      // (L or U)[sb rows, K] X_K over K = [0, r0) forward, [r0 + rn, n)
      // backward: waves (rh, kh) form rows rh*32.. of the product over the
      // 32-wide K slices q with q mod 2 == kh
      const int k_lo = sweep == 0 ? 0 : r0 + rn, k_hi = sweep == 0 ? r0 : n;
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
      for (int rt = 0; rt < 2; ++rt) row_ok[rt] = rh * NB + rt * 16 + li < rn;
      const int arow = r0 + rh * NB + li;
      // every load of a slice is issued ahead of its products (scheduling
      // barrier), so the 64 loads of a wave are in flight together
      for (int k0 = k_lo + 4 * KU * kh; k0 < k_hi; k0 += 8 * KU) {
        Slice<R, KU, PC> sl;
        sl.load(fr, fi, xrr, xir, (int)ld, arow, row_ok, k0, k_hi, lk, li);
        __builtin_amdgcn_sched_barrier(0);
        sl.product(pre, pim);
      }
      // T = X_sb - product (kh = 1 subtracts first, then kh = 0); stage blocks
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int idx = tid + 256 * j, r = idx / PC, c = idx % PC;
        const int o = r < rn ? (r0 * PC + idx) * (int)sizeof(R) : kOob;
        Tr[r][c] = BufLoad<R>::at(xrr, o);
        Ti[r][c] = BufLoad<R>::at(xir, o);
      }
      // the diagonal inverses as full matrices: unit lower (I + strict part)
      // forward, upper part backward; zero outside the block
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int idx = tid + 256 * j, r = idx % NB, c = idx / NB;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          R vr = pbr[m][j], vi = pbi[m][j];
          if (m != 1) {
            const int bn = m == 0 ? nf : ns;
            const bool keep = sweep == 0 ? c < r : c >= r;
            vr = keep ? vr : (sweep == 0 && c == r && r < bn ? R(1) : R(0));
            vi = keep ? vi : R(0);
          }
          Br[m][r][c] = vr;
          Bi[m][r][c] = vi;
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
                Tr[r][c] -= pre[rt][ct][q];
                Ti[r][c] -= pim[rt][ct][q];
              }
        }
        __syncthreads();
      }
      // triangular part: Y = M_f T_f; T_s -= C Y; X_s = M_s T_s, with M the
      // diagonal inverse (unit lower forward, upper backward) and C the
      // coupling block (rows of the second block, columns of the first)
      const int orow = (wave & 1) * 16, ocol = (wave >> 1) * 16 + li;
      if (nf > 0) {
        acc_t yre = acc_t{0, 0, 0, 0}, yim = acc_t{0, 0, 0, 0};
        tile_product<R, NB, PC>(Br[0], Bi[0], Tr + bf * NB, Ti + bf * NB, lane, wave, yre, yim);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = orow + Mfma<R>::row(lane, q);
          Yr[r][ocol] = yre[q];
          Yi[r][ocol] = yim[q];
          if (r < nf) {
            Xr[(int64_t)(r0 + bf * NB + r) * PC + ocol] = yre[q];
            Xi[(int64_t)(r0 + bf * NB + r) * PC + ocol] = yim[q];
          }
        }
        __syncthreads();
        if (ns > 0) {
          acc_t cre = acc_t{0, 0, 0, 0}, cim = acc_t{0, 0, 0, 0};
          tile_product<R, NB, PC>(Br[1], Bi[1], Yr, Yi, lane, wave, cre, cim);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = orow + Mfma<R>::row(lane, q);
            Tr[bs * NB + r][ocol] -= cre[q];
            Ti[bs * NB + r][ocol] -= cim[q];
          }
          __syncthreads();
        }
      }
      if (ns > 0) {
        acc_t yre = acc_t{0, 0, 0, 0}, yim = acc_t{0, 0, 0, 0};
        tile_product<R, NB, PC>(Br[2], Bi[2], Tr + bs * NB, Ti + bs * NB, lane, wave, yre, yim);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = orow + Mfma<R>::row(lane, q);
          if (r < ns) {
            Xr[(int64_t)(r0 + bs * NB + r) * PC + ocol] = yre[q];
            Xi[(int64_t)(r0 + bs * NB + r) * PC + ocol] = yim[q];
          }
        }
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

// The same sweeps with 128-row passes: the long product of a pass covers 128
// rows (each wave 32 rows over the whole K range), so X is re-read once per
// 128 factor rows instead of once per 64.  The pass is then solved as two
// 64-row halves in solve order; the second half first takes the product with
// the first half's new solutions (K = those 64 rows, read back from X), then
// the same three-block triangular step.  LDS: the 128-row T block, the
// diagonal inverse and coupling blocks (the second diagonal inverse waits in
// registers for the first one's LDS slot); solutions overwrite their T rows.
// In the long product the four waves multiply the same rows of X into their
// own factor rows, so X goes through LDS once per workgroup: strips of 4*KU
// rows, double-buffered in the space of the triangular blocks (unused
// then), the next strip loaded while the current one is multiplied; each
// complex product there takes three real MFMA products instead of four.
template <typename R, int NB, int PC, int KU>
__global__ void __launch_bounds__(256, 3) k_local_solve_multi_tall(
    const R* __restrict__ F, const int64_t* __restrict__ foff, const int* __restrict__ nsz,
    const int* __restrict__ lds, const int* __restrict__ perm, const int64_t* __restrict__ poff,
    const int* __restrict__ sub_dofs, const uint8_t* __restrict__ pou, const double2* __restrict__ v, int64_t vstride,
    const double2* __restrict__ vil, double2* __restrict__ z, int64_t zstride, R* __restrict__ xbuf, int64_t xchunk,
    int ncol, const int* __restrict__ active, const int* __restrict__ order) {
  static_assert(NB == 32 && PC == 32, "tile shape assumes 32 x 32 blocks");
  constexpr int SB = 4 * NB, HB = 2 * NB;   // rows per pass, rows per half
  typedef typename Mfma<R>::acc_t acc_t;
  // X strips in LDS: KS rows of X per strip, stored per column with the
  // rows in MFMA operand order (row 4u + lk at lk*KU + u, so a lane's KU
  // operands are contiguous), XLD entries per column (padded: the 16-byte
  // reads of a wave spread evenly over the banks)
  constexpr int KS = 4 * KU, XLD = KS + 4, EL = 16 / sizeof(R), LPT = KS * PC / EL / 256;
  static_assert(LPT >= 1 && KS * PC == LPT * EL * 256, "a strip is a whole number of 16-byte loads per thread");
  constexpr int kBlk = 2 * 2 * NB * (NB + 1), kStrip = 2 * 2 * PC * XLD;
  __shared__ R Tr[SB][PC + 1], Ti[SB][PC + 1];
  // [0] diagonal inverse, [1] coupling block of both planes; the strips
  __shared__ __attribute__((aligned(16))) R Bsh[kBlk > kStrip ? kBlk : kStrip];
  R(*Br)[NB][NB + 1] = reinterpret_cast<R(*)[NB][NB + 1]>(Bsh);
  R(*Bi)[NB][NB + 1] = reinterpret_cast<R(*)[NB][NB + 1]>(Bsh + 2 * NB * (NB + 1));
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
  const int tid = threadIdx.x, wave = tid >> 6;
  const __amdgpu_buffer_rsrc_t fr = plane_rsrc(Ar, ld * n * (int64_t)sizeof(R));
  const __amdgpu_buffer_rsrc_t fi = plane_rsrc(Ai, ld * n * (int64_t)sizeof(R));
  const __amdgpu_buffer_rsrc_t xrr = plane_rsrc(Xr, (int64_t)n * PC * sizeof(R));
  const __amdgpu_buffer_rsrc_t xir = plane_rsrc(Xi, (int64_t)n * PC * sizeof(R));

  // restrict and permute: X = P_s R_s v
  for (int base = tid; base < n * PC; base += 4 * 256) {
    double2 a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = base + u * 256;
      a[u] = make_double2(0.0, 0.0);
      if (idx < n * PC) {
        const int i = idx / PC, col = c0 + idx % PC;
        if (col < ncol)   // the interleaved copy: a row's columns in one contiguous read
          a[u] = vil ? vil[(int64_t)D[P[i]] * PC + idx % PC] : v[(int64_t)col * vstride + D[P[i]]];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = base + u * 256;
      if (idx < n * PC) {
        Xr[idx] = (R)a[u].x;
        Xi[idx] = (R)a[u].y;
      }
    }
  }
  __syncthreads();

  const int nsb = (n + SB - 1) / SB;
  for (int sweep = 0; sweep < 2; ++sweep) {
    for (int sq = 0; sq < nsb; ++sq) {
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      const int lane = tid & 63, li = lane & 15, lk = lane >> 4;
      const int sb = sweep == 0 ? sq : nsb - 1 - sq;
      const int r0 = sb * SB, rn = min(SB, n - r0);
      // the long product: wave w forms rows w*32.. of the pass over the whole
      // K range ([0, r0) forward, [r0 + rn, n) backward)
      const int k_lo = sweep == 0 ? 0 : r0 + rn, k_hi = sweep == 0 ? r0 : n;
      {
        // complex products by three real ones (Gauss): P1 = Ar Xr, P2 = Ai Xi,
        // P3 = (Ar + Ai)(Xr + Xi); Re = P1 - P2, Im = P3 - P1 - P2
        acc_t p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) p1[rt][ct] = p2[rt][ct] = p3[rt][ct] = acc_t{0, 0, 0, 0};
        bool row_ok[2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) row_ok[rt] = wave * NB + rt * 16 + li < rn;
        const int arow = r0 + wave * NB + li;
        typedef unsigned v4u __attribute__((ext_vector_type(4)));
        v4u gr[LPT], gi[LPT];   // the next strip in flight
        auto fetch = [&](int kb) {
#pragma unroll
          for (int l = 0; l < LPT; ++l) {
            const int e = (tid + 256 * l) * EL, kk = kb + e / PC;
            const int o = kk < k_hi ? (kk * PC + e % PC) * (int)sizeof(R) : kOob;
            gr[l] = __builtin_amdgcn_raw_buffer_load_b128(xrr, o, 0, 0);
            gi[l] = __builtin_amdgcn_raw_buffer_load_b128(xir, o, 0, 0);
          }
        };
        auto stash = [&](int buf) {
          R* sr = Bsh + buf * 2 * PC * XLD;
          R* si = sr + PC * XLD;
#pragma unroll
          for (int l = 0; l < LPT; ++l) {
            const int e = (tid + 256 * l) * EL, kk = e / PC, c = e % PC;
            const int pos = (kk & 3) * KU + (kk >> 2);
            R vr[EL], vi[EL];
            __builtin_memcpy(vr, &gr[l], 16);
            __builtin_memcpy(vi, &gi[l], 16);
#pragma unroll
            for (int j = 0; j < EL; ++j) {
              sr[(c + j) * XLD + pos] = vr[j];
              si[(c + j) * XLD + pos] = vi[j];
            }
          }
        };
        const int nst = (k_hi - k_lo + KS - 1) / KS;
        if (nst > 0) {
          fetch(k_lo);
          stash(0);
        }
        __syncthreads();
        for (int t = 0; t < nst; ++t) {
          const int kb = k_lo + t * KS;
          R ar[2][KU], ai[2][KU];
#pragma unroll
          for (int u = 0; u < KU; ++u) {
            const int kk = kb + 4 * u + lk;
            const int fo = (kk * (int)ld + arow) * (int)sizeof(R);
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
              const int o = (kk < k_hi && row_ok[rt]) ? fo + rt * 16 * (int)sizeof(R) : kOob;
              ar[rt][u] = BufLoad<R>::at(fr, o);
              ai[rt][u] = BufLoad<R>::at(fi, o);
            }
          }
          if (t + 1 < nst) fetch(kb + KS);
          const R* sr = Bsh + (t & 1) * 2 * PC * XLD;
          const R* si = sr + PC * XLD;
          R xr[2][KU], xi[2][KU];
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int u = 0; u < KU; ++u) {
              xr[ct][u] = sr[(ct * 16 + li) * XLD + lk * KU + u];
              xi[ct][u] = si[(ct * 16 + li) * XLD + lk * KU + u];
            }
#pragma unroll
          for (int u = 0; u < KU; ++u) {
            R as[2], xs[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              as[q] = ar[q][u] + ai[q][u];
              xs[q] = xr[q][u] + xi[q][u];
            }
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
              for (int ct = 0; ct < 2; ++ct) {
                p1[rt][ct] = Mfma<R>::op(ar[rt][u], xr[ct][u], p1[rt][ct]);
                p2[rt][ct] = Mfma<R>::op(ai[rt][u], xi[ct][u], p2[rt][ct]);
                p3[rt][ct] = Mfma<R>::op(as[rt], xs[ct], p3[rt][ct]);
              }
          }
          // the buffer written now was last read before the previous barrier
          if (t + 1 < nst) stash((t + 1) & 1);
          __syncthreads();
        }
        // T = X rows of the pass - product (each wave its own rows)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int idx = tid + 256 * j, r = idx / PC, c = idx % PC;
          const int o = r < rn ? (r0 * PC + idx) * (int)sizeof(R) : kOob;
          Tr[r][c] = BufLoad<R>::at(xrr, o);
          Ti[r][c] = BufLoad<R>::at(xir, o);
        }
        __syncthreads();
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
          for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int r = wave * NB + rt * 16 + Mfma<R>::row(lane, q), c = ct * 16 + li;
              Tr[r][c] -= p1[rt][ct][q] - p2[rt][ct][q];
              Ti[r][c] -= p3[rt][ct][q] - p1[rt][ct][q] - p2[rt][ct][q];
            }
        __syncthreads();
      }
      for (int half = 0; half < 2; ++half) {
        const int hb = sweep == 0 ? half : 1 - half;   // the half solved now (0: rows 0..63 of the pass)
        const int h0 = hb * HB, hn = min(HB, rn - h0);
        if (hn <= 0) continue;
        const int rh = wave & 1, kh = wave >> 1;
        if (half == 1) {
          // the other half's rows are solved (in X): T_h -= F[h rows, other rows] X_other
          const int o0 = (1 - hb) * HB, on = min(HB, rn - o0);
          const int klo = r0 + o0, khi = r0 + o0 + on;
          acc_t cre[2][2], cim[2][2];
#pragma unroll
          for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
              cre[rt][ct] = acc_t{0, 0, 0, 0};
              cim[rt][ct] = acc_t{0, 0, 0, 0};
            }
          bool row_ok[2];
#pragma unroll
          for (int rt = 0; rt < 2; ++rt) row_ok[rt] = rh * NB + rt * 16 + li < hn;
          const int arow = r0 + h0 + rh * NB + li;
          for (int k0 = klo + 4 * KU * kh; k0 < khi; k0 += 8 * KU) {
            Slice<R, KU, PC> sl;
            sl.load(fr, fi, xrr, xir, (int)ld, arow, row_ok, k0, khi, lk, li);
            __builtin_amdgcn_sched_barrier(0);
            sl.product(cre, cim);
          }
          for (int phase = 1; phase >= 0; --phase) {
            if (kh == phase) {
#pragma unroll
              for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                  for (int q = 0; q < 4; ++q) {
                    const int r = h0 + rh * NB + rt * 16 + Mfma<R>::row(lane, q), c = ct * 16 + li;
                    Tr[r][c] -= cre[rt][ct][q];
                    Ti[r][c] -= cim[rt][ct][q];
                  }
            }
            __syncthreads();
          }
        }
        // three-block triangular step of the half: blocks bf then bs (forward
        // 0 then 1, backward 1 then 0) within the half
        const int bf = sweep == 0 ? 0 : 1, bs = 1 - bf;
        const int nf = max(0, min(NB, hn - bf * NB)), ns = max(0, min(NB, hn - bs * NB));
        const int hr = r0 + h0;   // first row of the half in the matrix
        R pbr[3][4], pbi[3][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int idx = tid + 256 * j, r = idx % NB, c = idx / NB;
          const int rows[3] = {bf, bs, bs}, cols[3] = {bf, bf, bs};
          const int rlim[3] = {nf, ns, ns}, clim[3] = {nf, nf, ns};
#pragma unroll
          for (int m = 0; m < 3; ++m) {
            const bool in = r < rlim[m] && c < clim[m];
            const int o = in ? ((hr + cols[m] * NB + c) * (int)ld + hr + rows[m] * NB + r) * (int)sizeof(R) : kOob;
            R vr = BufLoad<R>::at(fr, o), vi = BufLoad<R>::at(fi, o);
            if (m != 1) {
              const int bn = m == 0 ? nf : ns;
              const bool keep = sweep == 0 ? c < r : c >= r;
              vr = keep ? vr : (sweep == 0 && c == r && r < bn ? R(1) : R(0));
              vi = keep ? vi : R(0);
            }
            pbr[m][j] = vr;
            pbi[m][j] = vi;
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int idx = tid + 256 * j, r = idx % NB, c = idx / NB;
          Br[0][r][c] = pbr[0][j];
          Bi[0][r][c] = pbi[0][j];
          Br[1][r][c] = pbr[1][j];
          Bi[1][r][c] = pbi[1][j];
        }
        __syncthreads();
        const int orow = (wave & 1) * 16, ocol = (wave >> 1) * 16 + li;
        R (*Tf)[PC + 1] = Tr + h0 + bf * NB;
        R (*Tfi)[PC + 1] = Ti + h0 + bf * NB;
        R (*Ts)[PC + 1] = Tr + h0 + bs * NB;
        R (*Tsi)[PC + 1] = Ti + h0 + bs * NB;
        if (nf > 0) {
          acc_t yre = acc_t{0, 0, 0, 0}, yim = acc_t{0, 0, 0, 0};
          tile_product<R, NB, PC>(Br[0], Bi[0], Tf, Tfi, lane, wave, yre, yim);
          __syncthreads();   // every wave has read T_f and M_f
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = orow + Mfma<R>::row(lane, q);
            Tf[r][ocol] = yre[q];
            Tfi[r][ocol] = yim[q];
            if (r < nf) {
              Xr[(int64_t)(hr + bf * NB + r) * PC + ocol] = yre[q];
              Xi[(int64_t)(hr + bf * NB + r) * PC + ocol] = yim[q];
            }
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {   // the second diagonal inverse takes M_f's place
            const int idx = tid + 256 * j, r = idx % NB, c = idx / NB;
            Br[0][r][c] = pbr[2][j];
            Bi[0][r][c] = pbi[2][j];
          }
          __syncthreads();
          if (ns > 0) {
            acc_t cre = acc_t{0, 0, 0, 0}, cim = acc_t{0, 0, 0, 0};
            tile_product<R, NB, PC>(Br[1], Bi[1], Tf, Tfi, lane, wave, cre, cim);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int r = orow + Mfma<R>::row(lane, q);
              Ts[r][ocol] -= cre[q];
              Tsi[r][ocol] -= cim[q];
            }
            __syncthreads();
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int idx = tid + 256 * j, r = idx % NB, c = idx / NB;
            Br[0][r][c] = pbr[2][j];
            Bi[0][r][c] = pbi[2][j];
          }
          __syncthreads();
        }
        if (ns > 0) {
          acc_t yre = acc_t{0, 0, 0, 0}, yim = acc_t{0, 0, 0, 0};
          tile_product<R, NB, PC>(Br[0], Bi[0], Ts, Tsi, lane, wave, yre, yim);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = orow + Mfma<R>::row(lane, q);
            if (r < ns) {
              Xr[(int64_t)(hr + bs * NB + r) * PC + ocol] = yre[q];
              Xi[(int64_t)(hr + bs * NB + r) * PC + ocol] = yim[q];
            }
          }
        }
        __syncthreads();
      }
    }
  }
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
                              double2* z, int64_t zstride, R* xbuf, int64_t sum_ns, int ncol, const int* active,
                              int ku, int rows) {
  if (a.n_sub == 0 || ncol == 0) return;
  const int nchunk = (ncol + kMultiPC - 1) / kMultiPC;
  const int64_t xchunk = 2 * sum_ns * kMultiPC;
  static_assert(kMultiPC == 32, "the interleaved copy holds 32 columns per unknown");
  const double2* vil = ncol <= kMultiPC ? a.vil : nullptr;
  // ku: 4-wide k steps per K slice of the long product; rows: rows per pass
  // over the factor (64, or 128 with 8-wide slices) -- tuning choices
  if (rows == 128)
    timed_launch(k_local_solve_multi_tall<R, kLuNB, kMultiPC, 8>, dim3(a.n_sub, nchunk), dim3(256), 0, st, F,
                 a.foff, a.nsz, a.lds, a.perm, a.poff, a.sub_dofs, a.pou, v, vstride, vil, z, zstride, xbuf, xchunk,
                 ncol, active, a.order);
  else if (ku == 4)
    timed_launch(k_local_solve_multi<R, kLuNB, kMultiPC, 4>, dim3(a.n_sub, nchunk), dim3(256), 0, st, F, a.foff,
                 a.nsz, a.lds, a.perm, a.poff, a.sub_dofs, a.pou, v, vstride, vil, z, zstride, xbuf, xchunk, ncol,
                 active, a.order);
  else
    timed_launch(k_local_solve_multi<R, kLuNB, kMultiPC, 8>, dim3(a.n_sub, nchunk), dim3(256), 0, st, F, a.foff,
                 a.nsz, a.lds, a.perm, a.poff, a.sub_dofs, a.pou, v, vstride, vil, z, zstride, xbuf, xchunk, ncol,
                 active, a.order);
}
template void launch_local_solve_multi<double>(hipStream_t, const LocalSolveArgs&, const double*, const double2*,
                                               int64_t, double2*, int64_t, double*, int64_t, int, const int*, int,
                                               int);
template void launch_local_solve_multi<float>(hipStream_t, const LocalSolveArgs&, const float*, const double2*,
                                              int64_t, double2*, int64_t, float*, int64_t, int, const int*, int,
                                              int);

int multi_chunk_cols() { return kMultiPC; }

}  // namespace mxw
