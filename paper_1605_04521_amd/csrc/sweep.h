// Building blocks of the blocked triangular sweeps on MFMA shared by the
// multi-column local solves and the left-looking LU: branch-free buffer loads,
// one K slice of a (rows x 32) += factor-strip x X product, and 32 x 32 tile
// products with matrices staged in LDS.
#pragma once

#include "device.h"

namespace mxw {

// Y = M T on MFMA for 32 x 32 M and T in LDS; each wave forms a 16 x 16
// tile (rows (wave & 1) * 16.., columns (wave >> 1) * 16..).
template <typename R, int NB, int PC>
__device__ __forceinline__ void tile_product(const R (*Br)[NB + 1], const R (*Bi)[NB + 1],
                                             const R (*Tr)[PC + 1], const R (*Ti)[PC + 1], int lane, int wave,
                                             typename Mfma<R>::acc_t& yre, typename Mfma<R>::acc_t& yim) {
  const int li = lane & 15, lk = lane >> 4;
  const int r = (wave & 1) * 16 + li, c = (wave >> 1) * 16 + li;
#pragma unroll
  for (int k0 = 0; k0 < NB; k0 += 4) {
    const int q = k0 + lk;
    const R mr = Br[r][q], mi = Bi[r][q];
    const R tr = Tr[q][c], ti = Ti[q][c];
    yre = Mfma<R>::op(mr, tr, yre);
    yre = Mfma<R>::op(-mi, ti, yre);
    yim = Mfma<R>::op(mr, ti, yim);
    yim = Mfma<R>::op(mi, tr, yim);
  }
}

// Buffer loads and stores: a descriptor per plane bounds every access (a load
// at or past the end of the plane reads 0, such a store is dropped).  Masked
// entries take the offset kOob, beyond every plane (a plane is at most
// 8192 x 8200 x 8 B < 1 GiB), so they need no branch around the access.
constexpr int kBufferFlags = 0x00020000;   // raw 32-bit buffer, gfx9 family
constexpr int kOob = 0x40000000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, kBufferFlags);
}

template <typename R>
struct BufLoad;
template <>
struct BufLoad<float> {
  __device__ __forceinline__ static float at(__amdgpu_buffer_rsrc_t r, int byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
  }
};
template <>
struct BufLoad<double> {
  __device__ __forceinline__ static double at(__amdgpu_buffer_rsrc_t r, int byte_off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
  }
};

template <typename R>
struct BufStore;
template <>
struct BufStore<float> {
  __device__ __forceinline__ static void at(__amdgpu_buffer_rsrc_t r, int byte_off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, byte_off, 0, 0);
  }
};
template <>
struct BufStore<double> {
  typedef int v2i __attribute__((ext_vector_type(2)));
  __device__ __forceinline__ static void at(__amdgpu_buffer_rsrc_t r, int byte_off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i, v), r, byte_off, 0, 0);
  }
};

// One K slice of the super-block product: 4*KU consecutive k (factor columns
// / rows of X), masked to zero past k_hi and past the super-block's rows,
// then accumulated on MFMA.
template <typename R, int KU, int PC>
struct Slice {
  R ar[2][KU], ai[2][KU], xr[2][KU], xi[2][KU];
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t fr, __amdgpu_buffer_rsrc_t fi,
                                       __amdgpu_buffer_rsrc_t xrr, __amdgpu_buffer_rsrc_t xir, int ld, int arow,
                                       const bool (&row_ok)[2], int k0, int k_hi, int lk, int li) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int kk = k0 + 4 * u + lk;
      const bool ok = kk < k_hi;
      const int fo = (kk * ld + arow) * (int)sizeof(R);
      const int xo = ok ? (kk * PC + li) * (int)sizeof(R) : kOob;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const int o = (ok && row_ok[rt]) ? fo + rt * 16 * (int)sizeof(R) : kOob;
        ar[rt][u] = BufLoad<R>::at(fr, o);
        ai[rt][u] = BufLoad<R>::at(fi, o);
      }
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        xr[ct][u] = BufLoad<R>::at(xrr, xo + ct * 16 * (int)sizeof(R));
        xi[ct][u] = BufLoad<R>::at(xir, xo + ct * 16 * (int)sizeof(R));
      }
    }
  }
  // The same products by three real ones (Gauss): P1 += Ar Xr, P2 += Ai Xi,
  // P3 += (Ar + Ai)(Xr + Xi); the product is P1 - P2 + i (P3 - P1 - P2).
  template <typename Acc>
  __device__ __forceinline__ void product3(Acc (&p1)[2][2], Acc (&p2)[2][2], Acc (&p3)[2][2]) const {
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
  }
  template <typename Acc>
  __device__ __forceinline__ void product(Acc (&pre)[2][2], Acc (&pim)[2][2]) const {
#pragma unroll
    for (int u = 0; u < KU; ++u)
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
};

}  // namespace mxw
