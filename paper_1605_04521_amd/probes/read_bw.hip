// Read-bandwidth probe (not part of the library): 2048 column-major complex
// n x n matrices (re and im planes, 113 GB), one workgroup per matrix, read
// in row strips of ROWS rows as the local-solve sweeps do, or contiguously:
// the streaming-read rate that launch shape reaches on the device.
// Build: hipcc --offload-arch=gfx950 -O3 -std=c++17 -Xclang -target-feature
//        -Xclang -packed-fp32-ops -o read_bw read_bw.hip
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
#define CHECK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s line %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

template <int ROWS>
__global__ void __launch_bounds__(256) strips(const double* __restrict__ F, int n, int64_t msize, double* out) {
  const double* A = F + (int64_t)blockIdx.x * msize;   // re plane, im plane follows at n*n
  constexpr int CG = 256 / ROWS;
  const int r = threadIdx.x % ROWS, cg = threadIdx.x / ROWS;
  double acc = 0.0;
  for (int b0 = 0; b0 + ROWS <= n; b0 += ROWS) {
    const double* cr = A + b0 + r;
    const double* ci = cr + (int64_t)n * n;
    int c = cg;
    for (; c + 7 * CG < n; c += 8 * CG) {
      double lr[8], li[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        lr[u] = cr[(int64_t)(c + u * CG) * n];
        li[u] = ci[(int64_t)(c + u * CG) * n];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += lr[u] * 1.0000001 + li[u];
    }
  }
  if (acc == 12345.678) out[0] = acc;
}

__global__ void __launch_bounds__(256) contig(const double* __restrict__ F, int64_t per, int64_t msize, double* out) {
  const double* A = F + (int64_t)blockIdx.x * msize;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < per; i += 256 * 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = (i + u * 256 < per) ? A[i + u * 256] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += t[u];
  }
  if (acc == 12345.678) out[0] = acc;
}

int main() {
  const int n = 1856, nmat = 2048;
  const int64_t msize = 2LL * n * n;   // re + im
  const size_t bytes = sizeof(double) * msize * nmat;
  printf("matrices %d of n=%d: %.1f GB\n", nmat, n, bytes / 1e9);
  double *F, *out;
  CHECK(hipMalloc(&F, bytes));
  CHECK(hipMalloc(&out, 64));
  CHECK(hipMemset(F, 0, bytes));
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  auto run = [&](const char* name, auto launch, double rb) {
    launch();
    hipDeviceSynchronize();
    hipEventRecord(a);
    for (int k = 0; k < 3; ++k) launch();
    hipEventRecord(b);
    hipEventSynchronize(b);
    float ms;
    hipEventElapsedTime(&ms, a, b);
    ms /= 3;
    printf("%-24s %8.2f ms  %7.0f GB/s\n", name, ms, rb / ms / 1e6);
  };
  const double rb = (double)bytes * ((n / 32) * 32.0 / n);
  run("strips 32 rows", [&] { hipLaunchKernelGGL(strips<32>, dim3(nmat), dim3(256), 0, 0, F, n, msize, out); }, (double)bytes);
  run("strips 64 rows", [&] { hipLaunchKernelGGL(strips<64>, dim3(nmat), dim3(256), 0, 0, F, n, msize, out); }, (double)bytes);
  run("strips 128 rows", [&] { hipLaunchKernelGGL(strips<128>, dim3(nmat), dim3(256), 0, 0, F, n, msize, out); }, (double)bytes);
  run("contiguous", [&] { hipLaunchKernelGGL(contig, dim3(nmat), dim3(256), 0, 0, F, msize, msize, out); }, (double)bytes);
  CHECK(hipGetLastError());
  (void)rb;
  return 0;
}
