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
             double *__restrict__ SDabx, double *__restrict__ Xabx) {
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
  Xabx[e] = -Xab[ex];
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

__global__ void __launch_bounds__(256) k_ny_combine(int r, NyCombineArgs a) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = tid64();
  if (e >= r2 * r2) return;
  const int l = (int)(e % r);
  int64_t t = e / r;
  const int k = (int)(t % r);
  t /= r;
  const int j = (int)(t % r);
  const int i = (int)(t / r);
  auto at = [&](const double *T, int x0, int x1, int x2, int x3) {
    return T[((int64_t)(x0 * r + x1) * r + x2) * r + x3];
  };
  auto bv = [&](int b, int x0, int x1, int x2, int x3) {
    const int bs = b == 0 ? 0 : 3 - b;  // block with the spins of i and j exchanged
    double pl = 0.0;
    const double *sd = a.sd[b] + (int64_t)(x0 * r + x1) * r2 + x3;
    const double *y = a.Y + (int64_t)x2 * r;
    for (int q = 0; q < r; ++q) pl += y[q] * sd[(int64_t)q * r];
    return 4.0 * (at(a.il[b], x0, x1, x2, x3) - at(a.il[bs], x1, x0, x2, x3) + pl -
                  2.0 * at(a.ir[b], x0, x1, x2, x3) + 2.0 * at(a.ir[bs], x1, x0, x2, x3) -
                  2.0 * at(a.pr[b], x0, x1, x2, x3));
  };
  a.Saa[e] -= bv(0, i, j, k, l) - bv(0, i, j, l, k);
  a.Sab[e] -= bv(1, i, j, k, l) - bv(2, i, j, l, k);
}

}  // namespace

hipError_t launch_ny_sources(int r, const double *g, const double *d2aa, const double *d2ab,
                             const double *Xab, const double *sigma, double *const src[7], hipStream_t s) {
  const int64_t n = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_ny_sources, grid_for(n), dim3(256), 0, s, r, g, d2aa, d2ab, Xab, sigma, src[0],
                     src[1], src[2], src[3], src[4], src[5], src[6]);
  return hipGetLastError();
}

hipError_t launch_ny_trace_y(int r, int64_t ld, const double *W0, const double *W5, double *Y, hipStream_t s) {
  hipLaunchKernelGGL(k_ny_trace_y, grid_for((int64_t)r * r), dim3(256), 0, s, r, ld, W0, W5, Y);
  return hipGetLastError();
}

hipError_t launch_ny_combine(int r, const NyCombineArgs &a, hipStream_t s) {
  const int64_t n = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_ny_combine, grid_for(n), dim3(256), 0, s, r, a);
  return hipGetLastError();
}

}  // namespace acse
