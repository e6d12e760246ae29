// Kernels of the hand-written adjoint (vector-Jacobian product) of the
// residual map: generic 4-index permutes into natural arrays or GEMM operand
// buffers, contractions of a 4-index tensor with an r x r matrix down to
// r x r, the particle-hole cotangent combination, the f-term rank-2 update,
// the adjoint of the fold of Eq. (2) and the projections of the gradients
// onto the symmetry subspaces of the inputs.
#include "vjp.h"

namespace acse {

__device__ inline int64_t vtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
static inline dim3 vgrid(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

struct VOutF64 {
  double *p;
  __device__ void put(int64_t i, double v) const { p[i] = v; }
};
struct VOutF64Acc {
  double *p;
  __device__ void put(int64_t i, double v) const { p[i] += v; }
};
struct VOutF32 {
  float *p;
  __device__ void put(int64_t i, double v) const { p[i] = (float)v; }
};
struct VOutBF16x3 {
  __bf16 *hi, *lo;
  __device__ void put(int64_t i, double v) const {
    const float f = (float)v;
    const __bf16 h = (__bf16)f;
    hi[i] = h;
    lo[i] = (__bf16)(f - (float)h);
  }
};

// dst[row][col] (rows x ld) = c1 src1[idx1] + c2 src2[idx2] for row, col < r^2,
// zero in the padding; row = (a, b), col = (c, d), idx = a s0 + b s1 + c s2 + d s3.
template <class O>
__global__ void k_permute4(PermArgs a, O out) {
  const int64_t r2 = (int64_t)a.r * a.r;
  const int64_t e = vtid();
  if (e >= a.rows * a.ld) return;
  const int64_t row = e / a.ld, col = e - row * a.ld;
  if (row >= r2 || col >= r2) {
    if (!a.accumulate) out.put(e, 0.0);
    return;
  }
  const int64_t i0 = row / a.r, i1 = row - i0 * a.r, i2 = col / a.r, i3 = col - i2 * a.r;
  double v = a.c1 * a.src1[i0 * a.s1[0] + i1 * a.s1[1] + i2 * a.s1[2] + i3 * a.s1[3]];
  if (a.src2) v += a.c2 * a.src2[i0 * a.s2[0] + i1 * a.s2[1] + i2 * a.s2[2] + i3 * a.s2[3]];
  out.put(e, v);
}

// out[x,y] (+)= sum_t c_t sum_{u,v} T_t[x sx + y sy + u su + v sv] M_t[u r + v]
// (one block per output element, fixed-order block reduction)
__global__ void __launch_bounds__(256)
k_contract42(int r, ContractArgs a, double *__restrict__ out, int accumulate) {
  __shared__ double red[256];
  const int x = blockIdx.x / r, y = blockIdx.x % r;
  double acc = 0.0;
  for (int t = 0; t < a.nterms; ++t) {
    const ContractTerm &q = a.term[t];
    const int64_t base = (int64_t)x * q.sx + (int64_t)y * q.sy;
    double s = 0.0;
    for (int uv = threadIdx.x; uv < r * r; uv += 256) {
      const int u = uv / r, v = uv - u * r;
      s += q.T[base + (int64_t)u * q.su + (int64_t)v * q.sv] * q.M[uv];
    }
    acc += q.c * s;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = accumulate ? out[blockIdx.x] + red[0] : red[0];
}

// Particle-hole cotangents from S-bar:
//   E1b = -(S_aa - S_aa[j,i,k,l] - S_aa[i,j,l,k] + S_aa[j,i,l,k]),  sym = S_ab + S_ab[j,i,l,k]
//   P+b = E1b - sym,  P-b = E1b + sym,  E3b = sym
__global__ void k_vjp_pe(int r, const double *__restrict__ Saa, const double *__restrict__ Sab,
                         double *__restrict__ Ppb, double *__restrict__ Pmb, double *__restrict__ E3b) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = vtid();
  if (e >= r2 * r2) return;
  const int l = e % r, k = (e / r) % r, j = (e / r2) % r, i = e / (r2 * r);
  const int64_t jikl = ((int64_t)j * r + i) * r2 + (int64_t)k * r + l;
  const int64_t ijlk = ((int64_t)i * r + j) * r2 + (int64_t)l * r + k;
  const int64_t jilk = ((int64_t)j * r + i) * r2 + (int64_t)l * r + k;
  const double e1 = -(Saa[e] - Saa[jikl] - Saa[ijlk] + Saa[jilk]);
  const double sym = Sab[e] + Sab[jilk];
  Ppb[e] = e1 - sym;
  Pmb[e] = e1 + sym;
  E3b[e] = sym;
}

// A_aa[k,p,a,b] += fb[k,b] g[p,a];  A_ab[k,p,a,b] -= fb[k,a] g[p,b]
__global__ void k_vjp_frank(int r, const double *__restrict__ fb, const double *__restrict__ g,
                            double *__restrict__ Abaa, double *__restrict__ Abab) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = vtid();
  if (e >= r2 * r2) return;
  const int b = e % r, a = (e / r) % r, p = (e / r2) % r, k = e / (r2 * r);
  Abaa[e] += fb[k * r + b] * g[p * r + a];
  Abab[e] -= fb[k * r + a] * g[p * r + b];
}

// Adjoint of the fold: K_s-bar = 1/2 (A_aa-bar - A_aa-bar(r<->s)) + 1/2 A_ab-bar;
// V-bar[p,r,q,s] = K_s-bar[p,q,r,s].
__global__ void k_vjp_fold_v(int r, const double *__restrict__ Abaa, const double *__restrict__ Abab,
                             double *__restrict__ Vb) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = vtid();
  if (e >= r2 * r2) return;
  const int s = e % r, q = (e / r) % r, rr = (e / r2) % r, p = e / (r2 * r);  // element (p,r,q,s)
  const int64_t pqrs = ((int64_t)p * r + q) * r2 + (int64_t)rr * r + s;
  const int64_t pqsr = ((int64_t)p * r + q) * r2 + (int64_t)s * r + rr;
  Vb[e] = 0.5 * (Abaa[pqrs] - Abaa[pqsr]) + 0.5 * Abab[pqrs];
}

// h-bar[p,r] = (sum_q K_s-bar[p,q,r,q] + sum_q K_s-bar[q,p,q,r]) / (N-1)
__global__ void k_vjp_fold_h(int r, double inv_nm1, const double *__restrict__ Abaa,
                             const double *__restrict__ Abab, double *__restrict__ hb) {
  const int e = (int)vtid();
  if (e >= r * r) return;
  const int p = e / r, rr = e % r;
  const int64_t r2 = (int64_t)r * r;
  auto ks = [&](int a, int b, int c, int d) {
    const int64_t x = ((int64_t)a * r + b) * r2 + (int64_t)c * r + d;
    const int64_t y = ((int64_t)a * r + b) * r2 + (int64_t)d * r + c;
    return 0.5 * (Abaa[x] - Abaa[y]) + 0.5 * Abab[x];
  };
  double acc = 0.0;
  for (int q = 0; q < r; ++q) acc += ks(p, q, rr, q) + ks(q, p, q, rr);
  hb[e] = acc * inv_nm1;
}

// Projections onto the symmetry subspaces of the inputs (scaled by c).
__global__ void k_proj_sym2(int r, double c, const double *__restrict__ x, double *__restrict__ out) {
  const int e = (int)vtid();
  if (e >= r * r) return;
  const int i = e / r, j = e % r;
  out[e] = c * 0.5 * (x[i * r + j] + x[j * r + i]);
}

__device__ inline int64_t ix4(int r, int a, int b, int c, int d) {
  const int64_t r2 = (int64_t)r * r;
  return ((int64_t)a * r + b) * r2 + (int64_t)c * r + d;
}

// 8-fold symmetry of (pq|rs)
__global__ void k_proj_v(int r, double c, const double *__restrict__ x, double *__restrict__ out) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = vtid();
  if (e >= r2 * r2) return;
  const int s = e % r, q2 = (e / r) % r, q = (e / r2) % r, p = e / (r2 * r);
  const double v = x[ix4(r, p, q, q2, s)] + x[ix4(r, q, p, q2, s)] + x[ix4(r, p, q, s, q2)] +
                   x[ix4(r, q, p, s, q2)] + x[ix4(r, q2, s, p, q)] + x[ix4(r, s, q2, p, q)] +
                   x[ix4(r, q2, s, q, p)] + x[ix4(r, s, q2, q, p)];
  out[e] = c * v / 8.0;
}

// alpha-alpha 2-RDM block: antisymmetric in both pairs, Hermitian
__global__ void k_proj_aa(int r, double c, const double *__restrict__ x, double *__restrict__ out) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = vtid();
  if (e >= r2 * r2) return;
  const int l = e % r, k = (e / r) % r, j = (e / r2) % r, i = e / (r2 * r);
  const double v = x[ix4(r, i, j, k, l)] - x[ix4(r, j, i, k, l)] - x[ix4(r, i, j, l, k)] +
                   x[ix4(r, j, i, l, k)] + x[ix4(r, k, l, i, j)] - x[ix4(r, l, k, i, j)] -
                   x[ix4(r, k, l, j, i)] + x[ix4(r, l, k, j, i)];
  out[e] = c * v / 8.0;
}

// alpha-beta 2-RDM block: Hermitian and symmetric under the pair exchange
__global__ void k_proj_ab(int r, double c, const double *__restrict__ x, double *__restrict__ out) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = vtid();
  if (e >= r2 * r2) return;
  const int l = e % r, k = (e / r) % r, j = (e / r2) % r, i = e / (r2 * r);
  const double v = x[ix4(r, i, j, k, l)] + x[ix4(r, k, l, i, j)] + x[ix4(r, j, i, l, k)] +
                   x[ix4(r, l, k, j, i)];
  out[e] = c * v / 4.0;
}

__global__ void k_identity(int r, double *__restrict__ I) {
  const int e = (int)vtid();
  if (e >= r * r) return;
  I[e] = (e / r == e % r) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
hipError_t launch_permute4(GemmPrec prec, const PermArgs &a, const OperandRef &out, hipStream_t s) {
  const int64_t n = a.rows * a.ld;
  if (a.accumulate) {
    if (prec != GEMM_F64) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_permute4<VOutF64Acc>), vgrid(n), dim3(256), 0, s, a,
                       VOutF64Acc{static_cast<double *>(out.hi)});
  } else if (prec == GEMM_F64) {
    hipLaunchKernelGGL((k_permute4<VOutF64>), vgrid(n), dim3(256), 0, s, a,
                       VOutF64{static_cast<double *>(out.hi)});
  } else if (prec == GEMM_F32) {
    hipLaunchKernelGGL((k_permute4<VOutF32>), vgrid(n), dim3(256), 0, s, a,
                       VOutF32{static_cast<float *>(out.hi)});
  } else {
    hipLaunchKernelGGL((k_permute4<VOutBF16x3>), vgrid(n), dim3(256), 0, s, a,
                       VOutBF16x3{static_cast<__bf16 *>(out.hi), static_cast<__bf16 *>(out.lo)});
  }
  return hipGetLastError();
}

hipError_t launch_contract42(int r, const ContractArgs &a, double *out, int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_contract42, dim3((unsigned)(r * r)), dim3(256), 0, s, r, a, out, accumulate);
  return hipGetLastError();
}

hipError_t launch_vjp_pe(int r, const double *Saa, const double *Sab, double *Ppb, double *Pmb,
                         double *E3b, hipStream_t s) {
  const int64_t n = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_vjp_pe, vgrid(n), dim3(256), 0, s, r, Saa, Sab, Ppb, Pmb, E3b);
  return hipGetLastError();
}

hipError_t launch_vjp_frank(int r, const double *fb, const double *g, double *Abaa, double *Abab,
                            hipStream_t s) {
  const int64_t n = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_vjp_frank, vgrid(n), dim3(256), 0, s, r, fb, g, Abaa, Abab);
  return hipGetLastError();
}

hipError_t launch_vjp_fold(int r, int N, const double *Abaa, const double *Abab, double *Vb_raw,
                           double *hb_raw, hipStream_t s) {
  const int64_t n = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_vjp_fold_v, vgrid(n), dim3(256), 0, s, r, Abaa, Abab, Vb_raw);
  hipLaunchKernelGGL(k_vjp_fold_h, vgrid((int64_t)r * r), dim3(256), 0, s, r, 1.0 / (N - 1), Abaa, Abab,
                     hb_raw);
  return hipGetLastError();
}

hipError_t launch_proj(ProjKind k, int r, double c, const double *x, double *out, hipStream_t s) {
  const int64_t n4 = (int64_t)r * r * r * r;
  switch (k) {
    case PROJ_SYM2: hipLaunchKernelGGL(k_proj_sym2, vgrid((int64_t)r * r), dim3(256), 0, s, r, c, x, out); break;
    case PROJ_V: hipLaunchKernelGGL(k_proj_v, vgrid(n4), dim3(256), 0, s, r, c, x, out); break;
    case PROJ_AA: hipLaunchKernelGGL(k_proj_aa, vgrid(n4), dim3(256), 0, s, r, c, x, out); break;
    case PROJ_AB: hipLaunchKernelGGL(k_proj_ab, vgrid(n4), dim3(256), 0, s, r, c, x, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_identity(int r, double *I, hipStream_t s) {
  hipLaunchKernelGGL(k_identity, vgrid((int64_t)r * r), dim3(256), 0, s, r, I);
  return hipGetLastError();
}

}  // namespace acse
