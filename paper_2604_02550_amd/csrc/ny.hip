// Element-wise and O(r^5) kernels of the Nakatsuji-Yasuda share of the
// residual map (Eq. (8); App. D, NY part).  The O(r^6) products run on the
// grouped FP64 MFMA GEMM, planned in ny_plan.h and launched from acse_api.hip.
#include "ny.h"

namespace acse {
namespace {

__device__ __forceinline__ int64_t tid64() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

__global__ void __launch_bounds__(256)
k_ny_sources(int r, const double *__restrict__ g, const double *__restrict__ d2aa,
             const double *__restrict__ d2ab, const double *__restrict__ Xab,
             const double *__restrict__ sig, double *__restrict__ Daa, double *__restrict__ Dab,
             double *__restrict__ Dabx, double *__restrict__ SDaa, double *__restrict__ SDab,
             double *__restrict__ SDabx, double *__restrict__ Xabx, int keep_d) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = tid64();
  if (e >= r2 * r2) return;
  const int s = (int)(e % r);
  int64_t t = e / r;
  const int c = (int)(t % r);  // third index
  t /= r;
  const int q = (int)(t % r);
  const int p = (int)(t / r);
  const int64_t ex = ((int64_t)(p * r + q) * r + s) * r + c;  // [p,q,s,c]
  Xabx[e] = -Xab[ex];
  if (keep_d) return;
  const double gpc = g[p * r + c], gqs = g[q * r + s], gps = g[p * r + s], gqc = g[q * r + c];
  const double daa = d2aa[e] - 0.5 * (gpc * gqs - gps * gqc);
  const double dab = d2ab[e] - 0.5 * gpc * gqs;
  const double dabx = -(d2ab[ex] - 0.5 * gps * gqc);
  const double sg = sig[c];
  Daa[e] = daa;
  Dab[e] = dab;
  Dabx[e] = dabx;
  SDaa[e] = sg * daa;
  SDab[e] = sg * dab;
  SDabx[e] = sg * dabx;
}

__global__ void __launch_bounds__(256) k_ny_unscramble(int64_t n, double *__restrict__ x, double *__restrict__ y) {
  const int64_t e = tid64();
  if (e >= n) return;
  const double a = x[e], b = y[e];
  x[e] = 0.5 * (a + b);
  y[e] = 0.5 * (a - b);
}

__global__ void __launch_bounds__(256)
k_ny_trace_y(int r, int64_t ld, const double *__restrict__ W0, const double *__restrict__ W5,
             double *__restrict__ Y) {
  const int64_t e = tid64();
  if (e >= (int64_t)r * r) return;
  const int k = (int)(e / r), a = (int)(e % r);
  double acc = 0.0;
  for (int p = 0; p < r; ++p) {
    const int64_t o = ((int64_t)p * r + k) * ld + (int64_t)p * r + a;
    acc += W0[o] + W5[o];
  }
  Y[e] = acc;
}

constexpr int kKB = 4;  // k values per thread in k_ny_bsum

// One block per (i,j) slab: Y and the slab SD(b)[i,j,:,:] in LDS, so the
// r-term sums of T_pl read LDS; the other terms are read along (k,l).
__global__ void __launch_bounds__(256) k_ny_bsum(int r, NyCombineArgs a) {
  extern __shared__ double lds[];
  const int rp = r + 1;
  double *ys = lds, *ss = lds + (int64_t)r * rp;
  const int64_t r2 = (int64_t)r * r;
  const int64_t ij = blockIdx.x;
  const int i = (int)(ij / r), j = (int)(ij % r);
  const int64_t base = ij * r2, jib = ((int64_t)j * r + i) * r2;
  for (int64_t x = threadIdx.x; x < r2; x += 256) ys[(x / r) * rp + x % r] = a.Y[x];
#pragma unroll 1
  for (int b = 0; b < 3; ++b) {
    const int bs = b == 0 ? 0 : 3 - b;  // block with the spins of i and j exchanged
    __syncthreads();
    for (int64_t x = threadIdx.x; x < r2; x += 256) ss[(x / r) * rp + x % r] = a.sd[b][base + x];
    __syncthreads();
    // a thread takes kKB consecutive k for one l: each slab value read from
    // LDS serves kKB sums (the Y reads are shared by the threads of a k group)
    const int nkb = (r + kKB - 1) / kKB;
    for (int task = threadIdx.x; task < r * nkb; task += 256) {
      const int l = task % r, k0 = (task / r) * kKB;
      double pl[kKB];
#pragma unroll
      for (int u = 0; u < kKB; ++u) pl[u] = 0.0;
      for (int q = 0; q < r; ++q) {
        const double sv = ss[q * rp + l];
#pragma unroll
        for (int u = 0; u < kKB; ++u) pl[u] += ys[min(k0 + u, r - 1) * rp + q] * sv;
      }
#pragma unroll
      for (int u = 0; u < kKB; ++u) {
        const int k = k0 + u;
        if (k >= r) break;
        const int64_t x = (int64_t)k * r + l;
        a.B[b][base + x] = 4.0 * (a.il[b][base + x] - a.il[bs][jib + x] + pl[u] - 2.0 * a.ir[b][base + x] +
                                  2.0 * a.ir[bs][jib + x] - 2.0 * a.pr[b][base + x]);
      }
    }
  }
}

// One block per (i,j) slab: S_aa -= B0 - B0^T, S_ab -= B1 - B2^T, T the
// exchange of k and l within the slab, read from LDS.
__global__ void __launch_bounds__(256) k_ny_sub(int r, NyCombineArgs a) {
  extern __shared__ double lds[];
  const int rp = r + 1;
  double *t0 = lds, *t2 = lds + (int64_t)r * rp;
  const int64_t r2 = (int64_t)r * r;
  const int64_t base = (int64_t)blockIdx.x * r2;
  for (int64_t x = threadIdx.x; x < r2; x += 256) {
    const int k = (int)(x / r), l = (int)(x % r);
    t0[k * rp + l] = a.B[0][base + x];
    t2[k * rp + l] = a.B[2][base + x];
  }
  __syncthreads();
  for (int64_t x = threadIdx.x; x < r2; x += 256) {
    const int k = (int)(x / r), l = (int)(x % r);
    a.Saa[base + x] -= t0[k * rp + l] - t0[l * rp + k];
    a.Sab[base + x] -= a.B[1][base + x] - t2[l * rp + k];
  }
}

}  // namespace

hipError_t launch_ny_sources(int r, const double *g, const double *d2aa, const double *d2ab,
                             const double *Xab, const double *sigma, double *const src[7], bool keep_d,
                             hipStream_t s) {
  const int64_t n = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_ny_sources, grid_for(n), dim3(256), 0, s, r, g, d2aa, d2ab, Xab, sigma, src[0],
                     src[1], src[2], src[3], src[4], src[5], src[6], keep_d ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_ny_unscramble(int64_t n, double *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_ny_unscramble, grid_for(n), dim3(256), 0, s, n, x, y);
  return hipGetLastError();
}

hipError_t launch_ny_trace_y(int r, int64_t ld, const double *W0, const double *W5, double *Y, hipStream_t s) {
  hipLaunchKernelGGL(k_ny_trace_y, grid_for((int64_t)r * r), dim3(256), 0, s, r, ld, W0, W5, Y);
  return hipGetLastError();
}

hipError_t launch_ny_combine(int r, const NyCombineArgs &a, hipStream_t s) {
  const int64_t r2 = (int64_t)r * r;
  const size_t lds = (size_t)2 * r * (r + 1) * sizeof(double);
  for (const void *k : {reinterpret_cast<const void *>(&k_ny_bsum), reinterpret_cast<const void *>(&k_ny_sub)}) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ny_bsum, dim3((unsigned)r2), dim3(256), lds, s, r, a);
  hipLaunchKernelGGL(k_ny_sub, dim3((unsigned)r2), dim3(256), lds, s, r, a);
  return hipGetLastError();
}

}  // namespace acse
