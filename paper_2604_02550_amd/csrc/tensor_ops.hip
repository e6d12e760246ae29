// O(r^4) and O(r^5) kernels of the ACSE residual path: the fold of the
// reduced Hamiltonian, the cumulant operand W and its particle-hole
// relayouts, one-index transforms, the residual assembly, FP64 reductions
// and the step (axpy, trace restoration, 1-RDM contraction, energy).
//
// Spatial 4-index arrays are row-major [p][q][r][s] with n4 = r^4 elements.
// GEMM operands are [rows][ld] matrices (rows = pair index, ld >= padded K)
// in the contraction precision; the F64/F32/BF16x3 variants are selected by
// the OpT template parameter (BF16x3 writes a hi and a lo plane).
#include "tensor_ops.h"

namespace acse {

// ---------------------------------------------------------------------------
// Operand element writers
// ---------------------------------------------------------------------------
struct OutF64 {
  double *p;
  __device__ void put(int64_t i, double v) const { p[i] = v; }
};
struct OutF32 {
  float *p;
  __device__ void put(int64_t i, double v) const { p[i] = (float)v; }
};
struct OutBF16x3 {
  __bf16 *hi, *lo;
  __device__ void put(int64_t i, double v) const {
    const float f = (float)v;
    const __bf16 h = (__bf16)f;
    hi[i] = h;
    lo[i] = (__bf16)(f - (float)h);
  }
};

__device__ inline int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// ---------------------------------------------------------------------------
// Fold of Eq. (2): X_A blocks of the reduced Hamiltonian
//   K_s[p,q,r,s] = (pr|qs) + (h_pr d_qs + h_qs d_pr)/(N-1)
//   A_aa = 1/2 (K_s[k,l,r,s] - K_s[k,l,s,r]),  A_ab = 1/2 K_s[k,l,r,s]
// (pr|qs) = V[p,r,q,s]; the exchange term uses (ks|lr) = (lr|ks) = V[l,r,k,s]
// so both reads run along s.
// ---------------------------------------------------------------------------
__global__ void k_fold(int r, double inv_nm1, const double *__restrict__ h,
                       const double *__restrict__ V, double *__restrict__ Aaa,
                       double *__restrict__ Aab) {
  const int64_t n4 = (int64_t)r * r * r * r;
  const int64_t e = gtid();
  if (e >= n4) return;
  const int s = e % r, rr = (e / r) % r, l = (e / ((int64_t)r * r)) % r, k = e / ((int64_t)r * r * r);
  const int64_t r2 = (int64_t)r * r, r3 = r2 * r;
  const double dir = V[k * r3 + rr * r2 + l * r + s] +
                     ((s == l ? h[k * r + rr] : 0.0) + (k == rr ? h[l * r + s] : 0.0)) * inv_nm1;
  const double exc = V[l * r3 + rr * r2 + k * r + s] +
                     ((rr == l ? h[k * r + s] : 0.0) + (k == s ? h[l * r + rr] : 0.0)) * inv_nm1;
  Aaa[e] = 0.5 * (dir - exc);
  Aab[e] = 0.5 * dir;
}

// ---------------------------------------------------------------------------
// Cumulant operand W = Gamma2 - 2/3 Gamma1^Gamma1 (Eq. (7), App. C):
//   W_aa[a,b,c,d] = 2 d2aa - 2/3 (g_ac g_bd - g_ad g_bc)
//   W_ab[a,b,c,d] = 2 d2ab - 2/3 g_ac g_bd
// ---------------------------------------------------------------------------
__device__ inline double w_aa(const double *d2aa, const double *g, int r, int a, int b, int c, int d) {
  const int64_t r2 = (int64_t)r * r;
  return 2.0 * d2aa[((int64_t)a * r + b) * r2 + (int64_t)c * r + d] -
         (2.0 / 3.0) * (g[a * r + c] * g[b * r + d] - g[a * r + d] * g[b * r + c]);
}
__device__ inline double w_ab(const double *d2ab, const double *g, int r, int a, int b, int c, int d) {
  const int64_t r2 = (int64_t)r * r;
  return 2.0 * d2ab[((int64_t)a * r + b) * r2 + (int64_t)c * r + d] -
         (2.0 / 3.0) * g[a * r + c] * g[b * r + d];
}

__global__ void k_w_natural(int r, const double *__restrict__ g, const double *__restrict__ d2aa,
                            const double *__restrict__ d2ab, double *__restrict__ Waa,
                            double *__restrict__ Wab) {
  const int64_t n4 = (int64_t)r * r * r * r;
  const int64_t e = gtid();
  if (e >= n4) return;
  const int d = e % r, c = (e / r) % r, b = (e / ((int64_t)r * r)) % r, a = e / ((int64_t)r * r * r);
  Waa[e] = w_aa(d2aa, g, r, a, b, c, d);
  Wab[e] = w_ab(d2ab, g, r, a, b, c, d);
}

// Particle-hole B operands, rows (j,l) / (i,l), columns (p,s):
//   Rp[(j,l),(p,s)] = W_aa[j,p,s,l] - W_ab[j,p,l,s]
//   Rm[(j,l),(p,s)] = W_aa[j,p,s,l] + W_ab[j,p,l,s]
//   R3[(i,l),(p,s)] = W_ab[i,p,s,l]
// Columns >= r^2 (K padding) are written as zero.
template <class O>
__global__ void k_w_ph(int r, int ld, const double *__restrict__ g, const double *__restrict__ d2aa,
                       const double *__restrict__ d2ab, O Rp, O Rm, O R3) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = gtid();
  if (e >= r2 * ld) return;
  const int col = e % ld;
  const int row = e / ld;
  if (col >= r2) {
    Rp.put(e, 0.0); Rm.put(e, 0.0); R3.put(e, 0.0);
    return;
  }
  const int j = row / r, l = row % r, p = col / r, s = col % r;
  const double a = w_aa(d2aa, g, r, j, p, s, l);
  const double b = w_ab(d2ab, g, r, j, p, l, s);
  Rp.put(e, a - b);
  Rm.put(e, a + b);
  R3.put(e, w_ab(d2ab, g, r, j, p, s, l));
}

// pp A operands: the unnormalised 2-RDM blocks Gamma2 = 2 2D (the factor 2
// is applied as the GEMM alpha), copied into the padded operand layout.
template <class O>
__global__ void k_d_operand(int r, int ld, const double *__restrict__ d2aa,
                            const double *__restrict__ d2ab, O Daa, O Dab) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = gtid();
  if (e >= r2 * ld) return;
  const int col = e % ld;
  const int64_t row = e / ld;
  if (col >= r2) { Daa.put(e, 0.0); Dab.put(e, 0.0); return; }
  Daa.put(e, d2aa[row * r2 + col]);
  Dab.put(e, d2ab[row * r2 + col]);
}

// Zero the K-padding columns [r^2, ld) of rows [0, r^2) of an operand whose
// producer writes only the first r^2 columns.
template <class O>
__global__ void k_zero_kpad(int r, int ld, O out) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t w = ld - r2;
  const int64_t e = gtid();
  if (w <= 0 || e >= r2 * w) return;
  out.put((e / w) * ld + r2 + e % w, 0.0);
}

// ---------------------------------------------------------------------------
// f[k,s] = sum_pr (A_aa[k,p,r,s] - A_ab[k,p,s,r]) g[p,r]: partial over r per
// (k,p,s), then a reduction over p.
// ---------------------------------------------------------------------------
__global__ void k_f_partial(int r, const double *__restrict__ Aaa, const double *__restrict__ Aab,
                            const double *__restrict__ g, double *__restrict__ part) {
  const int64_t r3 = (int64_t)r * r * r;
  const int64_t e = gtid();
  if (e >= r3) return;
  const int s = e % r, p = (e / r) % r, k = e / ((int64_t)r * r);
  const int64_t base = (int64_t)k * r3 + (int64_t)p * r * r;
  double acc = 0.0;
  for (int rr = 0; rr < r; ++rr)
    acc += (Aaa[base + (int64_t)rr * r + s] - Aab[base + (int64_t)s * r + rr]) * g[p * r + rr];
  part[e] = acc;  // [k][p][s]
}
__global__ void k_f_reduce(int r, const double *__restrict__ part, double *__restrict__ f) {
  const int e = (int)gtid();
  if (e >= r * r) return;
  const int k = e / r, s = e % r;
  double acc = 0.0;
  for (int p = 0; p < r; ++p) acc += part[((int64_t)k * r + p) * r + s];
  f[e] = acc;
}

// ---------------------------------------------------------------------------
// Mode product:  out[a, x, b] = alpha * sum_y M(x, y) * (c1 in1 + c2 in2)[a, y, b]
// in* contiguous [A][r][Bn]; M(x,y) = g[x*r+y] or g[y*r+x] (transposed);
// output element address (a/adiv)*so1 + (a%adiv)*so0 + x*sx + b*sb.
// A block owns NCOL consecutive (a,b) columns; the r x NCOL input panel and
// M are staged in LDS so every input element is read from HBM once.
// ---------------------------------------------------------------------------
constexpr int kModeCols = 64;

template <class O>
__global__ void __launch_bounds__(256)
k_mode(ModeArgs m, O out) {
  extern __shared__ double mode_smem[];
  const int r = m.r;
  const int ldm = r + 1;
  double *Ms = mode_smem;              // [r][r+1]
  double *T = mode_smem + r * ldm;     // [r][kModeCols]
  const int64_t ncols = (int64_t)m.A * m.Bn;
  const int64_t c0 = (int64_t)blockIdx.x * kModeCols;
  const int nc = (int)min<int64_t>(kModeCols, ncols - c0);
  for (int e = threadIdx.x; e < r * r; e += 256) {
    const int x = e / r, y = e % r;
    Ms[x * ldm + y] = m.transpose_m ? m.g[y * r + x] : m.g[x * r + y];
  }
  const bool along_b = m.Bn >= kModeCols;
  for (int e = threadIdx.x; e < r * kModeCols; e += 256) {
    int y, c;
    if (along_b) { y = e / kModeCols; c = e % kModeCols; } else { c = e / r; y = e % r; }
    double v = 0.0;
    if (c < nc) {
      const int64_t col = c0 + c;
      const int64_t a = col / m.Bn, b = col % m.Bn;
      const int64_t off = (a * r + y) * m.Bn + b;
      v = m.c1 * m.in1[off];
      if (m.in2) v += m.c2 * m.in2[off];
    }
    T[y * kModeCols + c] = v;
  }
  __syncthreads();
  // lanes run along the columns when the output is contiguous in the column
  // index, else along x
  for (int e = threadIdx.x; e < r * kModeCols; e += 256) {
    int x, c;
    if (m.out_cols_fast) { x = e / kModeCols; c = e % kModeCols; } else { c = e / r; x = e % r; }
    if (c >= nc) continue;
    double acc = 0.0;
    for (int y = 0; y < r; ++y) acc += Ms[x * ldm + y] * T[y * kModeCols + c];
    const int64_t col = c0 + c;
    const int64_t a = col / m.Bn, b = col % m.Bn;
    const int64_t off = (a / m.adiv) * m.so1 + (a % m.adiv) * m.so0 + (int64_t)x * m.sx + b * m.sb;
    out.put(off, m.alpha * acc);
  }
}

// ---------------------------------------------------------------------------
// pp B operands and the G2 tensors (fold of the f and H terms):
//   G2_aa[k,l,r,s] = H_aa[k,l,r,s] - H_aa[l,k,r,s]
//                    + f[k,r] d_ls - f[k,s] d_lr - f[l,r] d_ks + f[l,s] d_kr
//   G2_ab[k,l,r,s] = H_ab[k,l,r,s] + H_ab[l,k,s,r] + f[k,r] d_ls + f[l,s] d_kr
//   Bpp = A - G2 (operand precision, padded), G2 kept in FP64.
// ---------------------------------------------------------------------------
template <class O>
__global__ void k_g2(int r, int ld, const double *__restrict__ Aaa, const double *__restrict__ Aab,
                     const double *__restrict__ Haa, const double *__restrict__ Hab,
                     const double *__restrict__ f, double *__restrict__ G2aa,
                     double *__restrict__ G2ab, O Baa, O Bab) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = gtid();
  if (e >= r2 * ld) return;
  const int col = e % ld;
  const int row = e / ld;
  if (col >= r2) { Baa.put(e, 0.0); Bab.put(e, 0.0); return; }
  const int k = row / r, l = row % r, rr = col / r, s = col % r;
  const int64_t nat = (int64_t)row * r2 + col;
  double gaa = Haa[nat] - Haa[((int64_t)l * r + k) * r2 + col];
  if (l == s) gaa += f[k * r + rr];
  if (l == rr) gaa -= f[k * r + s];
  if (k == s) gaa -= f[l * r + rr];
  if (k == rr) gaa += f[l * r + s];
  double gab = Hab[nat] + Hab[((int64_t)l * r + k) * r2 + (int64_t)s * r + rr];
  if (l == s) gab += f[k * r + rr];
  if (k == rr) gab += f[l * r + s];
  G2aa[nat] = gaa;
  G2ab[nat] = gab;
  Baa.put(e, Aaa[nat] - gaa);
  Bab.put(e, Aab[nat] - gab);
}

// ---------------------------------------------------------------------------
// Assembly of S (before the (ij)<->(kl) exchange), FP64:
//   S_aa = Z_aa - (g_il t_jk - g_jl t_ik - g_ik t_jl + g_jk t_il)
//               - (E1[i,j,k,l] - E1[j,i,k,l] - E1[i,j,l,k] + E1[j,i,l,k])
//   S_ab = Z_ab + g_jl t_ik + g_ik t_jl
//               - (E2[i,j,k,l] + E2[j,i,l,k] - E3[i,j,k,l] - E3[j,i,l,k])
// with E1 = P+ + P-, E2 = P+ - P- (all stored [i,j,k,l]).
// ---------------------------------------------------------------------------
__global__ void k_assemble(int r, const double *__restrict__ g, const double *__restrict__ t,
                           const double *__restrict__ Zaa, const double *__restrict__ Zab,
                           const double *__restrict__ Pp, const double *__restrict__ Pm,
                           const double *__restrict__ E3, double *__restrict__ Saa,
                           double *__restrict__ Sab) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t n4 = r2 * r2;
  const int64_t e = gtid();
  if (e >= n4) return;
  const int l = e % r, k = (e / r) % r, j = (e / r2) % r, i = e / (r2 * r);
  const int64_t ijkl = e;
  const int64_t jikl = ((int64_t)j * r + i) * r2 + (int64_t)k * r + l;
  const int64_t ijlk = ((int64_t)i * r + j) * r2 + (int64_t)l * r + k;
  const int64_t jilk = ((int64_t)j * r + i) * r2 + (int64_t)l * r + k;
  const double pp_ijkl = Pp[ijkl], pm_ijkl = Pm[ijkl];
  const double pp_jilk = Pp[jilk], pm_jilk = Pm[jilk];
  const double e1 = (pp_ijkl + pm_ijkl) - (Pp[jikl] + Pm[jikl]) - (Pp[ijlk] + Pm[ijlk]) + (pp_jilk + pm_jilk);
  const double e2 = (pp_ijkl - pm_ijkl) + (pp_jilk - pm_jilk) - E3[ijkl] - E3[jilk];
  const double gt_aa = g[i * r + l] * t[j * r + k] - g[j * r + l] * t[i * r + k] -
                       g[i * r + k] * t[j * r + l] + g[j * r + k] * t[i * r + l];
  const double gt_ab = g[j * r + l] * t[i * r + k] + g[i * r + k] * t[j * r + l];
  Saa[e] = Zaa[e] - gt_aa - e1;
  Sab[e] = Zab[e] + gt_ab - e2;
}

// Out = S + sigma S^T ((ij)<->(kl)) with S = S' + C^T; optional masked copy; per-block partial
// sums of 2 Out_aa^2 + 4 Out_ab^2 (deterministic two-pass reduction).
__global__ void __launch_bounds__(256)
k_finish(int r, double sigma, const double *__restrict__ Saa, const double *__restrict__ Sab,
         const double *__restrict__ Caa, const double *__restrict__ Cab,
         double *__restrict__ Oaa, double *__restrict__ Oab, ActiveBits active,
         double *__restrict__ Maa, double *__restrict__ Mab, double *__restrict__ partial) {
  __shared__ double red[256];
  const int64_t r2 = (int64_t)r * r;
  const int64_t n4 = r2 * r2;
  const int64_t e = gtid();
  double acc = 0.0;
  if (e < n4) {
    const int64_t row = e / r2, col = e % r2;
    const int64_t tr = col * r2 + row;
    // S = S' + C^T where C (stored [k,l,i,j]) is the separable gamma-gamma term
    const double a = (Saa[e] + Caa[tr]) + sigma * (Saa[tr] + Caa[e]);
    const double b = (Sab[e] + Cab[tr]) + sigma * (Sab[tr] + Cab[e]);
    Oaa[e] = a;
    Oab[e] = b;
    acc = 2.0 * a * a + 4.0 * b * b;
    if (Maa) {
      const int l = e % r, k = (e / r) % r, j = (e / r2) % r, i = e / (r2 * r);
      auto act = [&](int q) { return (active.w[q >> 6] >> (q & 63)) & 1ull; };
      const bool all_active = act(i) && act(j) && act(k) && act(l);
      Maa[e] = all_active ? 0.0 : a;
      Mab[e] = all_active ? 0.0 : b;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Sum of n partials in a fixed order by one block; writes out[0].
__global__ void __launch_bounds__(256)
k_reduce_sum(int64_t n, const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t q = threadIdx.x; q < n; q += 256) acc += part[q];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// t[j,k] = sum_x (W_aa[j,x] A_aa[k,x] + 2 W_ab[j,x] A_ab[k,x]),  x = (p,r,s) in [0, r^3).
// Block b reduces its own x range; each thread owns up to 3 register tiles of
// 4 x 4 (j,k) outputs; x slabs of kTChunk are staged x-major in LDS so a
// thread reads its 4 j's and 4 k's as consecutive doubles.
// ---------------------------------------------------------------------------
constexpr int kTChunk = 32;
constexpr int kTBlocks = 256;

__global__ void __launch_bounds__(256)
k_t_partial(int r, const double *__restrict__ Waa, const double *__restrict__ Aaa,
            const double *__restrict__ Wab, const double *__restrict__ Aab,
            double *__restrict__ part) {
  extern __shared__ double t_smem[];
  const int rp = (r + 3) & ~3;
  double *sWa = t_smem, *sAa = sWa + kTChunk * rp, *sWb = sAa + kTChunk * rp, *sAb = sWb + kTChunk * rp;
  const int64_t X = (int64_t)r * r * r;
  const int64_t per = (X + gridDim.x - 1) / gridDim.x;
  const int64_t x0 = (int64_t)blockIdx.x * per, x1 = min(X, x0 + per);
  const int nb = rp / 4;
  double acc[3][16];
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[u][q] = 0.0;
  for (int64_t xc = x0; xc < x1; xc += kTChunk) {
    for (int e = threadIdx.x; e < kTChunk * rp; e += 256) {
      const int c = e % kTChunk, j = e / kTChunk;
      const int64_t x = xc + c;
      const bool ok = (j < r) && (x < x1);
      const int64_t o = (int64_t)j * X + x;
      sWa[c * rp + j] = ok ? Waa[o] : 0.0;
      sAa[c * rp + j] = ok ? Aaa[o] : 0.0;
      sWb[c * rp + j] = ok ? Wab[o] : 0.0;
      sAb[c * rp + j] = ok ? Aab[o] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int q = threadIdx.x + u * 256;
      if (q >= nb * nb) break;
      const int jb = (q / nb) * 4, kb = (q % nb) * 4;
      for (int c = 0; c < kTChunk; ++c) {
        double wa[4], aa[4], wb[4], ab[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          wa[v] = sWa[c * rp + jb + v]; aa[v] = sAa[c * rp + kb + v];
          wb[v] = sWb[c * rp + jb + v]; ab[v] = sAb[c * rp + kb + v];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[u][a * 4 + b] += wa[a] * aa[b] + 2.0 * wb[a] * ab[b];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int q = threadIdx.x + u * 256;
    if (q >= nb * nb) break;
    const int jb = (q / nb) * 4, kb = (q % nb) * 4;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (jb + a < r && kb + b < r)
          part[(int64_t)blockIdx.x * r * r + (jb + a) * r + kb + b] = acc[u][a * 4 + b];
  }
}

// t[j,k] = sum over the per-block partials of k_t_partial.
__global__ void k_t_reduce(int r, int nsplit_total, const double *__restrict__ part,
                           double *__restrict__ t) {
  const int e = (int)gtid();
  if (e >= r * r) return;
  double acc = 0.0;
  for (int q = 0; q < nsplit_total; ++q) acc += part[(int64_t)q * r * r + e];
  t[e] = acc;
}

// ---------------------------------------------------------------------------
// Energy E = 2 sum K_s[p,q,r,s] (d2aa + d2ab)[p,q,r,s]  (per-block partials)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_energy_partial(int r, double inv_nm1, const double *__restrict__ h, const double *__restrict__ V,
                 const double *__restrict__ d2aa, const double *__restrict__ d2ab,
                 double *__restrict__ partial) {
  __shared__ double red[256];
  const int64_t r2 = (int64_t)r * r;
  const int64_t n4 = r2 * r2;
  const int64_t e = gtid();
  double acc = 0.0;
  if (e < n4) {
    const int s = e % r, rr = (e / r) % r, q = (e / r2) % r, p = e / (r2 * r);
    double ks = V[(int64_t)p * r2 * r + (int64_t)rr * r2 + (int64_t)q * r + s];
    if (q == s) ks += h[p * r + rr] * inv_nm1;
    if (p == rr) ks += h[q * r + s] * inv_nm1;
    acc = 2.0 * ks * (d2aa[e] + d2ab[e]);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// Step pieces (FP64)
// ---------------------------------------------------------------------------
// traces[0..1] = (Tr d2aa, Tr d2ab) in a fixed order (one block).
__global__ void __launch_bounds__(256)
k_traces(int r, const double *__restrict__ d2aa, const double *__restrict__ d2ab,
         double *__restrict__ traces) {
  __shared__ double ra[256], rb[256];
  const int64_t r2 = (int64_t)r * r;
  double a = 0.0, b = 0.0;
  for (int64_t q = threadIdx.x; q < r2; q += 256) {
    const int64_t d = q * r2 + q;  // element (p,q,p,q) at row = col = p*r+q
    a += d2aa[d];
    b += d2ab[d];
  }
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) { ra[threadIdx.x] += ra[threadIdx.x + w]; rb[threadIdx.x] += rb[threadIdx.x + w]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { traces[0] = ra[0]; traces[1] = rb[0]; }
}

// out = d2 + eps U (new blocks into the workspace copies)
__global__ void k_axpy2(int64_t n, double eps, const double *__restrict__ aa, const double *__restrict__ ab,
                        const double *__restrict__ Uaa, const double *__restrict__ Uab,
                        double *__restrict__ oaa, double *__restrict__ oab) {
  const int64_t e = gtid();
  if (e >= n) return;
  oaa[e] = aa[e] + eps * Uaa[e];
  oab[e] = ab[e] + eps * Uab[e];
}

// d2 = new * (trace_in / trace_new) per block; traces = [in_aa, in_ab, new_aa, new_ab]
__global__ void k_rescale(int64_t n, const double *__restrict__ traces, const double *__restrict__ naa,
                          const double *__restrict__ nab, double *__restrict__ d2aa,
                          double *__restrict__ d2ab) {
  const int64_t e = gtid();
  if (e >= n) return;
  const double sa = traces[0] / traces[2], sb = traces[1] / traces[3];
  d2aa[e] = naa[e] * sa;
  d2ab[e] = nab[e] * sb;
}

// gamma[p,r] = 2/(N-1) sum_q (d2aa[p,q,r,q] + d2ab[p,q,r,q])
__global__ void k_contract_1rdm(int r, double two_over_nm1, const double *__restrict__ d2aa,
                                const double *__restrict__ d2ab, double *__restrict__ g) {
  const int e = (int)gtid();
  if (e >= r * r) return;
  const int p = e / r, rr = e % r;
  const int64_t r2 = (int64_t)r * r;
  double acc = 0.0;
  for (int q = 0; q < r; ++q) {
    const int64_t o = ((int64_t)p * r + q) * r2 + (int64_t)rr * r + q;
    acc += d2aa[o] + d2ab[o];
  }
  g[e] = two_over_nm1 * acc;
}

__global__ void k_fill(int64_t n, double v, double *__restrict__ p) {
  const int64_t e = gtid();
  if (e < n) p[e] = v;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
static inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_fold(int r, int N, const double *h, const double *V, double *Aaa, double *Aab,
                       hipStream_t s) {
  const int64_t n4 = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_fold, grid_for(n4), dim3(256), 0, s, r, 1.0 / (N - 1), h, V, Aaa, Aab);
  return hipGetLastError();
}

hipError_t launch_w_natural(int r, const double *g, const double *d2aa, const double *d2ab,
                            double *Waa, double *Wab, hipStream_t s) {
  const int64_t n4 = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_w_natural, grid_for(n4), dim3(256), 0, s, r, g, d2aa, d2ab, Waa, Wab);
  return hipGetLastError();
}

template <class O> static O make_out(const OperandRef &o);
template <> OutF64 make_out<OutF64>(const OperandRef &o) { return {static_cast<double *>(o.hi)}; }
template <> OutF32 make_out<OutF32>(const OperandRef &o) { return {static_cast<float *>(o.hi)}; }
template <> OutBF16x3 make_out<OutBF16x3>(const OperandRef &o) {
  return {static_cast<__bf16 *>(o.hi), static_cast<__bf16 *>(o.lo)};
}

#define ACSE_DISPATCH_OUT(prec, CALL)                    \
  do {                                                   \
    if ((prec) == GEMM_F64) { using O = OutF64; CALL; }  \
    else if ((prec) == GEMM_F32) { using O = OutF32; CALL; } \
    else { using O = OutBF16x3; CALL; }                  \
  } while (0)

hipError_t launch_w_ph(GemmPrec prec, int r, int ld, const double *g, const double *d2aa,
                       const double *d2ab, const OperandRef &Rp, const OperandRef &Rm,
                       const OperandRef &R3, hipStream_t s) {
  const int64_t n = (int64_t)r * r * ld;
  ACSE_DISPATCH_OUT(prec, hipLaunchKernelGGL((k_w_ph<O>), grid_for(n), dim3(256), 0, s, r, ld, g, d2aa,
                                             d2ab, make_out<O>(Rp), make_out<O>(Rm), make_out<O>(R3)));
  return hipGetLastError();
}

hipError_t launch_d_operand(GemmPrec prec, int r, int ld, const double *d2aa, const double *d2ab,
                            const OperandRef &Daa, const OperandRef &Dab, hipStream_t s) {
  const int64_t n = (int64_t)r * r * ld;
  ACSE_DISPATCH_OUT(prec, hipLaunchKernelGGL((k_d_operand<O>), grid_for(n), dim3(256), 0, s, r, ld,
                                             d2aa, d2ab, make_out<O>(Daa), make_out<O>(Dab)));
  return hipGetLastError();
}

hipError_t launch_zero_kpad(GemmPrec prec, int r, int ld, const OperandRef &o, hipStream_t s) {
  const int64_t n = (int64_t)r * r * (ld - (int64_t)r * r);
  if (n <= 0) return hipSuccess;
  ACSE_DISPATCH_OUT(prec, hipLaunchKernelGGL((k_zero_kpad<O>), grid_for(n), dim3(256), 0, s, r, ld,
                                             make_out<O>(o)));
  return hipGetLastError();
}

hipError_t launch_f(int r, const double *Aaa, const double *Aab, const double *g, double *part,
                    double *f, hipStream_t s) {
  const int64_t r3 = (int64_t)r * r * r;
  hipLaunchKernelGGL(k_f_partial, grid_for(r3), dim3(256), 0, s, r, Aaa, Aab, g, part);
  hipLaunchKernelGGL(k_f_reduce, grid_for((int64_t)r * r), dim3(256), 0, s, r, part, f);
  return hipGetLastError();
}

size_t mode_lds_bytes(int r) { return (size_t)(r * (r + 1) + r * kModeCols) * sizeof(double); }

hipError_t launch_mode(GemmPrec prec, const ModeArgs &m, const OperandRef &out, hipStream_t s) {
  if (m.r > kModeMaxR) return hipErrorInvalidValue;
  const int64_t ncols = (int64_t)m.A * m.Bn;
  const dim3 grid((unsigned)((ncols + kModeCols - 1) / kModeCols));
  const size_t lds = mode_lds_bytes(m.r);
  ACSE_DISPATCH_OUT(prec, {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_mode<O>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_mode<O>), grid, dim3(256), lds, s, m, make_out<O>(out));
  });
  return hipGetLastError();
}

hipError_t launch_g2(GemmPrec prec, int r, int ld, const double *Aaa, const double *Aab,
                     const double *Haa, const double *Hab, const double *f, double *G2aa,
                     double *G2ab, const OperandRef &Baa, const OperandRef &Bab, hipStream_t s) {
  const int64_t n = (int64_t)r * r * ld;
  ACSE_DISPATCH_OUT(prec, hipLaunchKernelGGL((k_g2<O>), grid_for(n), dim3(256), 0, s, r, ld, Aaa, Aab,
                                             Haa, Hab, f, G2aa, G2ab, make_out<O>(Baa), make_out<O>(Bab)));
  return hipGetLastError();
}

hipError_t launch_assemble(int r, const double *g, const double *t, const double *Zaa,
                           const double *Zab, const double *Pp, const double *Pm, const double *E3,
                           double *Saa, double *Sab, hipStream_t s) {
  const int64_t n4 = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_assemble, grid_for(n4), dim3(256), 0, s, r, g, t, Zaa, Zab, Pp, Pm, E3, Saa, Sab);
  return hipGetLastError();
}

hipError_t launch_finish(int r, double sigma, const double *Saa, const double *Sab,
                         const double *Caa, const double *Cab, double *Oaa, double *Oab,
                         const ActiveBits &active, double *Maa, double *Mab, double *partial,
                         double *sum_out, hipStream_t s) {
  const int64_t n4 = (int64_t)r * r * r * r;
  const int64_t nb = (n4 + 255) / 256;
  hipLaunchKernelGGL(k_finish, dim3((unsigned)nb), dim3(256), 0, s, r, sigma, Saa, Sab, Caa, Cab,
                     Oaa, Oab, active, Maa, Mab, partial);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, nb, partial, sum_out);
  return hipGetLastError();
}

int64_t finish_partials(int r) { return ((int64_t)r * r * r * r + 255) / 256; }

hipError_t launch_t_reduce(int r, int nparts, const double *part, double *t, hipStream_t s) {
  hipLaunchKernelGGL(k_t_reduce, grid_for((int64_t)r * r), dim3(256), 0, s, r, nparts, part, t);
  return hipGetLastError();
}

int t_partial_blocks() { return kTBlocks; }

hipError_t launch_t(int r, const double *Waa, const double *Aaa, const double *Wab,
                    const double *Aab, double *part, double *t, hipStream_t s) {
  const int rp = (r + 3) & ~3;
  const size_t lds = (size_t)4 * kTChunk * rp * sizeof(double);
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_t_partial),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_t_partial, dim3(kTBlocks), dim3(256), lds, s, r, Waa, Aaa, Wab, Aab, part);
  return launch_t_reduce(r, kTBlocks, part, t, s);
}

hipError_t launch_energy(int r, int N, const double *h, const double *V, const double *d2aa,
                         const double *d2ab, double *partial, double *E_out, hipStream_t s) {
  const int64_t n4 = (int64_t)r * r * r * r;
  const int64_t nb = (n4 + 255) / 256;
  hipLaunchKernelGGL(k_energy_partial, dim3((unsigned)nb), dim3(256), 0, s, r, 1.0 / (N - 1), h, V,
                     d2aa, d2ab, partial);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, nb, partial, E_out);
  return hipGetLastError();
}

hipError_t launch_traces(int r, const double *d2aa, const double *d2ab, double *traces, hipStream_t s) {
  hipLaunchKernelGGL(k_traces, dim3(1), dim3(256), 0, s, r, d2aa, d2ab, traces);
  return hipGetLastError();
}

hipError_t launch_axpy2(int r, double eps, const double *aa, const double *ab, const double *Uaa,
                        const double *Uab, double *oaa, double *oab, hipStream_t s) {
  const int64_t n4 = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_axpy2, grid_for(n4), dim3(256), 0, s, n4, eps, aa, ab, Uaa, Uab, oaa, oab);
  return hipGetLastError();
}

hipError_t launch_rescale(int r, const double *traces, const double *naa, const double *nab,
                          double *d2aa, double *d2ab, hipStream_t s) {
  const int64_t n4 = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_rescale, grid_for(n4), dim3(256), 0, s, n4, traces, naa, nab, d2aa, d2ab);
  return hipGetLastError();
}

hipError_t launch_contract_1rdm(int r, int N, const double *d2aa, const double *d2ab, double *g,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_contract_1rdm, grid_for((int64_t)r * r), dim3(256), 0, s, r, 2.0 / (N - 1),
                     d2aa, d2ab, g);
  return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double v, double *p, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, grid_for(n), dim3(256), 0, s, n, v, p);
  return hipGetLastError();
}

}  // namespace acse
