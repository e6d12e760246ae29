// O(r^4) and O(r^5) kernels of the ACSE residual path: the fold of the
// reduced Hamiltonian, the cumulant operand W and its particle-hole
// relayouts, one-index transforms, the residual assembly, FP64 reductions
// and the step (axpy, trace restoration, 1-RDM contraction, energy).
//
// Spatial 4-index arrays are row-major [p][q][r][s] with n4 = r^4 elements.
// GEMM operands are [rows][ld] matrices (rows = pair index, ld >= padded K)
// in the contraction precision; the F64/F32/BF16x3 variants are selected by
// the OpT template parameter (BF16x3 writes a hi and a lo plane).
#include <algorithm>

#include "tensor_ops.h"

namespace acse {

// ---------------------------------------------------------------------------
// Operand element writers
// ---------------------------------------------------------------------------
struct OutF64 {
  double *p;
  __device__ void put(int64_t i, double v) const { p[i] = v; }
};
struct OutF64Acc {
  double *p;
  __device__ void put(int64_t i, double v) const { p[i] += v; }
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

// Unconditional load from a clamped, always valid address: staging loops issue
// a whole batch of these before consuming any, so the loads overlap (a guarded
// load would make the compiler wait for each one before the next).
__device__ inline double ld_ok(const double *__restrict__ p, int64_t off, bool ok) {
  return p[ok ? off : 0];
}

// LDS bytes one workgroup may allocate on gfx950 (160 KiB per CU).
constexpr size_t kMaxLds = 160 * 1024;

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
// Columns >= r^2 (K padding) are written as zero.  One block per (j,p): the
// 2-RDM slabs d2aa[j,p,:,:], d2ab[j,p,:,:] (contiguous) and rows j, p of g are
// staged in LDS (row stride r + 1), and the block writes the r x r column
// segment (p, :) of the r rows (j, :) in contiguous runs; the block with
// p = r - 1 also zeroes the padding columns of those rows.
constexpr int kWphU = 4;

template <class O>
__global__ void __launch_bounds__(256)
k_w_ph(int r, int ld, const double *__restrict__ g, const double *__restrict__ d2aa,
       const double *__restrict__ d2ab, O Rp, O Rm, O R3) {
  extern __shared__ double wph_smem[];
  constexpr int NT = 256, U = kWphU;
  const int r2 = r * r, RP = r + 1;
  const int j = blockIdx.x / r, p = blockIdx.x - (blockIdx.x / r) * r;
  double *Sa = wph_smem, *Sb = wph_smem + r * RP, *gj = wph_smem + 2 * r * RP, *gp = gj + r;
  const int64_t src = (int64_t)blockIdx.x * r2;  // d2[j,p,:,:]
  const int tid = threadIdx.x;
  for (int base = 0; base < r2; base += NT * U) {
    double va[U], vb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * NT + tid;
      va[u] = ld_ok(d2aa, src + e, e < r2);
      vb[u] = ld_ok(d2ab, src + e, e < r2);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * NT + tid;
      if (e < r2) {
        const int c = e / r, d = e - (e / r) * r;
        Sa[c * RP + d] = va[u];
        Sb[c * RP + d] = vb[u];
      }
    }
  }
  for (int e = tid; e < r; e += NT) {
    gj[e] = g[j * r + e];
    gp[e] = g[p * r + e];
  }
  __syncthreads();
  constexpr double c23 = 2.0 / 3.0;
  for (int e = tid; e < r2; e += NT) {
    const int l = e / r, s = e - (e / r) * r;
    // W_aa[j,p,s,l], W_ab[j,p,l,s], W_ab[j,p,s,l]
    const double waa = 2.0 * Sa[s * RP + l] - c23 * (gj[s] * gp[l] - gj[l] * gp[s]);
    const double wab = 2.0 * Sb[l * RP + s] - c23 * gj[l] * gp[s];
    const double w3 = 2.0 * Sb[s * RP + l] - c23 * gj[s] * gp[l];
    const int64_t o = ((int64_t)j * r + l) * ld + (int64_t)p * r + s;
    Rp.put(o, waa - wab);
    Rm.put(o, waa + wab);
    R3.put(o, w3);
  }
  if (p == r - 1) {
    const int pad = ld - r2;
    for (int e = tid; e < r * pad; e += NT) {
      const int l = e / pad, c = e - (e / pad) * pad;
      const int64_t o = ((int64_t)j * r + l) * ld + r2 + c;
      Rp.put(o, 0.0);
      Rm.put(o, 0.0);
      R3.put(o, 0.0);
    }
  }
}

// pp A operands, packed by the pair symmetries of the 2-RDM blocks (the factor
// of the unnormalised Gamma2 = 2 2D and the 2 of the exchange are GEMM alphas):
//   D_aa[(i<j), (r<s)] = d2aa[i,j,r,s]                       (antisymmetric pairs)
//   D_S [(i<=j), (r<=s)] = d2ab[i,j,r,s] + d2ab[i,j,s,r]  (r < s),  d2ab[i,j,r,r]
//   D_A [(i<j), (r<s)]  = d2ab[i,j,r,s] - d2ab[i,j,s,r]
// One block per unordered pair i <= j stages the two 2-RDM rows in LDS; the
// K padding of each written row is zeroed.
template <class O>
__global__ void __launch_bounds__(256)
k_d_operand(int r, int ld_lt, int ld_le, const double *__restrict__ d2aa,
            const double *__restrict__ d2ab, O Daa, O DS, O DA) {
  extern __shared__ double dop_smem[];
  const int r2 = r * r;
  int i, j;
  unpair_le(r, blockIdx.x, i, j);
  const int64_t src = ((int64_t)i * r + j) * r2;
  double *ra = dop_smem, *rb = dop_smem + r2;
  for (int e = threadIdx.x; e < r2; e += 256) {
    ra[e] = d2aa[src + e];
    rb[e] = d2ab[src + e];
  }
  __syncthreads();
  const int nle = npair_le(r), nlt = npair_lt(r);
  const int64_t rowS = (int64_t)blockIdx.x * ld_le;
  for (int q = threadIdx.x; q < ld_le; q += 256) {
    double v = 0.0;
    if (q < nle) {
      int a, b;
      unpair_le(r, q, a, b);
      v = a == b ? rb[a * r + a] : rb[a * r + b] + rb[b * r + a];
    }
    DS.put(rowS + q, v);
  }
  if (i < j) {
    const int64_t rowA = (int64_t)pair_lt(r, i, j) * ld_lt;
    for (int q = threadIdx.x; q < ld_lt; q += 256) {
      double va = 0.0, vd = 0.0;
      if (q < nlt) {
        int a, b;
        unpair_lt(r, q, a, b);
        va = ra[a * r + b];
        vd = rb[a * r + b] - rb[b * r + a];
      }
      Daa.put(rowA + q, va);
      DA.put(rowA + q, vd);
    }
  }
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
#pragma unroll 8
  for (int rr = 0; rr < r; ++rr)
    acc += (Aaa[base + (int64_t)rr * r + s] - Aab[base + (int64_t)s * r + rr]) * g[p * r + rr];
  part[e] = acc;  // [k][p][s]
}
// f[k,s] = sum_p part[k,p,s]: one wavefront per output, lanes over p,
// fixed-order shuffle reduction.
__global__ void __launch_bounds__(256)
k_f_reduce(int r, const double *__restrict__ part, double *__restrict__ f) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= r * r) return;
  const int k = e / r, s = e % r;
  double acc = 0.0;
  for (int p = lane; p < r; p += 64) acc += part[((int64_t)k * r + p) * r + s];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) f[e] = acc;
}

// ---------------------------------------------------------------------------
// Mode product:  out[a, x, b] = alpha * sum_y M(x, y) * (c1 in1 + c2 in2)[a, y, b]
// in* contiguous [A][r][Bn]; M(x,y) = g[x*r+y] or g[y*r+x] (transposed);
// output element address (a/adiv)*so1 + (a%adiv)*so0 + x*sx + b*sb.
//
// A small dense contraction (2r flops per output) over a long stream of
// columns (a,b), bound by HBM.  It runs on the FP64 MFMA (16x16x4): M is the
// A operand and stays in registers for the whole kernel (wave w holds row
// blocks w and w + 4 of M, one fragment per K step of 4); the input panel of
// COLS columns is staged in LDS and feeds the B fragments (one double per lane
// per MFMA, so LDS traffic stays far below its bandwidth).  Persistent blocks
// walk the panels; the next panel's global loads are in flight into registers
// while the current one is multiplied.  Results are stored from the
// accumulators (16 consecutive columns per row and instruction).
// ---------------------------------------------------------------------------
constexpr int kStage = 8;  // global loads in flight per thread in LDS staging loops

typedef double mode_d4 __attribute__((ext_vector_type(4)));

template <int COLS>
struct ModeShape {
  static constexpr int LDT = COLS + 1;   // odd panel row stride (conflict-free deposits)
  static constexpr int YS = 256 / COLS;  // rows per pass of the strided loader
  static constexpr int PF = 8;           // prefetched elements per thread (r * COLS <= 2048)
  static constexpr int CB = COLS / 16;   // MFMA column blocks per panel
};

// KS: K steps of 4 (a compile-time trip count, 4 KS >= r; the A fragments and
// panel rows beyond r are zero), so the MFMA chain is straight-line code.
template <class O, int COLS, int NRB, bool HAS2, int KS>
__global__ void __launch_bounds__(256)
k_mode(ModeArgs m, O out, int npanels) {
  using S = ModeShape<COLS>;
  constexpr int KSMAX = KS;
  extern __shared__ double mode_smem[];
  const int r = m.r;
  // two [4 KS][LDT] input panels (double buffer); rows >= r stay zero
  double *const T0 = mode_smem;
  double *const T1 = mode_smem + 4 * KS * S::LDT;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int Bn = (int)m.Bn;
  const int ncols = (int)(m.A * m.Bn);   // A * Bn <= r^4 < 2^31
  const double c1 = m.c1, c2 = m.c2;
  const double *in2 = m.in2;

  // A fragments: lane holds M(x = 16 rb + lr, y = 4 ks + lk)
  double afr[NRB][KSMAX];
#pragma unroll
  for (int q = 0; q < NRB; ++q) {
    const int x = (wave + 4 * q) * 16 + lr;
#pragma unroll
    for (int ks = 0; ks < KSMAX; ++ks) {
      const int y = ks * 4 + lk;
      const bool ok = x < r && y < r;
      const double v = ld_ok(m.g, m.transpose_m ? (int64_t)y * r + x : (int64_t)x * r + y, ok);
      afr[q][ks] = ok ? v : 0.0;
    }
  }
  for (int e = r * S::LDT + tid; e < 4 * KS * S::LDT; e += 256) T0[e] = T1[e] = 0.0;

  // flat walk (Bn == 1): element f of the panel is column f / r, row f % r
  const int dc = 256 / r, dy = 256 - (256 / r) * r;
  const int c_first = tid / r, y_first = tid - (tid / r) * r;

  double v1[S::PF], v2[HAS2 ? S::PF : 1];
  auto fetch = [&](int p) {
    const int c0 = p * COLS;
    const int nc = min(COLS, ncols - c0);
    if (Bn == 1) {
      const int64_t base = (int64_t)c0 * r;
      const int tot = nc * r;
#pragma unroll
      for (int k = 0; k < S::PF; ++k) {
        const int f = tid + k * 256;
        v1[k] = ld_ok(m.in1, base + f, f < tot);
        if constexpr (HAS2) v2[k] = ld_ok(in2, base + f, f < tot);
      }
    } else {
      const int c = tid % COLS;
      const bool okc = c < nc;
      const int col = c0 + (okc ? c : 0);
      const int a = col / Bn, b = col - (col / Bn) * Bn;
      const int64_t off0 = (int64_t)a * r * Bn + b;
#pragma unroll
      for (int k = 0; k < S::PF; ++k) {
        const int y = tid / COLS + k * S::YS;
        const bool ok = okc && y < r;
        v1[k] = ld_ok(m.in1, off0 + (int64_t)y * Bn, ok);
        if constexpr (HAS2) v2[k] = ld_ok(in2, off0 + (int64_t)y * Bn, ok);
      }
    }
  };
  auto combine = [&](int k) {
    if constexpr (HAS2) return c1 * v1[k] + c2 * v2[k];
    else return c1 * v1[k];
  };
  auto deposit = [&](int p, double *T) {
    const int nc = min(COLS, ncols - p * COLS);
    if (Bn == 1) {
      const int tot = nc * r;
      int c = c_first, y = y_first;
#pragma unroll
      for (int k = 0; k < S::PF; ++k) {
        const int f = tid + k * 256;
        if (c < COLS) T[y * S::LDT + c] = f < tot ? combine(k) : 0.0;
        c += dc;
        y += dy;
        if (y >= r) { y -= r; ++c; }
      }
    } else {
      const int c = tid % COLS;
#pragma unroll
      for (int k = 0; k < S::PF; ++k) {
        const int y = tid / COLS + k * S::YS;
        if (y < r) T[y * S::LDT + c] = c < nc ? combine(k) : 0.0;
      }
    }
  };

  // iteration k multiplies the panel in buffer k & 1 while the next panel's
  // loads are in flight; those land in buffer (k + 1) & 1 (last read in k - 1)
  // before the one barrier of the iteration.
  int p = blockIdx.x;
  int cur = 0;
  fetch(p);
  deposit(p, T0);
  __syncthreads();
  const double alpha = m.alpha;
  const int adiv = (int)m.adiv;
  for (;;) {
    const int pn = p + (int)gridDim.x;
    const bool more = pn < npanels;
    if (more) fetch(pn);
    const double *T = cur ? T1 : T0;
    mode_d4 acc[NRB][S::CB];
#pragma unroll
    for (int q = 0; q < NRB; ++q)
#pragma unroll
      for (int cb = 0; cb < S::CB; ++cb) acc[q][cb] = mode_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KSMAX; ++ks) {
      const double *tp = T + (ks * 4 + lk) * S::LDT + lr;
#pragma unroll
      for (int cb = 0; cb < S::CB; ++cb) {
        const double bfr = tp[cb * 16];
#pragma unroll
        for (int q = 0; q < NRB; ++q)
          acc[q][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[q][ks], bfr, acc[q][cb], 0, 0, 0);
      }
    }
    // store: accumulator item v of lane l is row lk + 4v of the block, column lr
    const int c0 = p * COLS;
    const int nc = min(COLS, ncols - c0);
#pragma unroll
    for (int cb = 0; cb < S::CB; ++cb) {
      const int cc = cb * 16 + lr;
      if (cc < nc) {
        const int col = c0 + cc;
        const int a = col / Bn, b = col - (col / Bn) * Bn;
        const int a1 = a / adiv, a0 = a - (a / adiv) * adiv;
        const int64_t base = (int64_t)a1 * m.so1 + (int64_t)a0 * m.so0 + (int64_t)b * m.sb;
#pragma unroll
        for (int q = 0; q < NRB; ++q)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int x = (wave + 4 * q) * 16 + lk + 4 * v;
            if (x < r) out.put(base + (int64_t)x * m.sx, alpha * acc[q][cb][v]);
          }
      }
    }
    if (!more) break;
    deposit(pn, cur ? T0 : T1);
    __syncthreads();
    cur ^= 1;
    p = pn;
  }
}

// ---------------------------------------------------------------------------
// The three ph A operands in one pass over the two input blocks (r <= 56):
//   L+[(k,i),(p,s)] = sum_r g[i,r] (X_aa + X_ab)[k,p,r,s]
//   L-[(k,i),(p,s)] = sum_r g[i,r] (X_aa - X_ab)[k,p,r,s]
//   L3[(k,j),(p,s)] = sum_r g[j,r] X_ab[k,p,s,r]
// i.e. per slab (k,p) three r x r products with g.  Persistent blocks walk the
// r^2 slabs; the two input slabs are staged in LDS (rows r.., columns r.. of
// the staging area zero; the next slab's loads are in flight in registers
// during the MFMAs), g is the FP64 MFMA A operand held in registers (wave w:
// output rows 16w..16w+15), and the output rows (k,i) get the 16-column runs
// (p, s).  The block that handles p = r - 1 also zeroes the K padding of the
// r rows (k, .) of all three operands.  With fpart set, the slab's partial of
// f[k,s] = sum_pr (X_aa[k,p,r,s] - X_ab[k,p,s,r]) g[p,r] (the sum over r, in
// the order of k_f_partial) is written too, [k][p][s].  LDS row stride: >= 4 KS and = 2 mod 4,
// which keeps the transposed reads of X_ab conflict-free.
// ---------------------------------------------------------------------------
static inline int lops_rp(int ks) { return 4 * ks + 2; }

template <class O, int KS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_lops(int r, int ld, int rp, const double *__restrict__ g, const double *__restrict__ Xaa,
       const double *__restrict__ Xab, O Lp, O Lm, O L3, int nslab, double *__restrict__ fpart) {
  constexpr int CB = (4 * KS + 15) / 16;   // 16-column output blocks (and 16-row blocks)
  constexpr int NR = CB * 16;              // staged rows (>= 4 KS, >= r)
  constexpr int PF = (4 * KS * 4 * KS + 255) / 256;  // prefetched elements per thread per slab
  extern __shared__ double lops_smem[];
  double *SA = lops_smem, *SB = lops_smem + NR * rp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int r2 = r * r;
  double afr[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int x = wave * 16 + lr, y = ks * 4 + lk;
    const bool ok = x < r && y < r;
    const double v = ld_ok(g, (int64_t)x * r + y, ok);
    afr[ks] = ok ? v : 0.0;
  }
  for (int e = tid; e < 2 * NR * rp; e += 256) lops_smem[e] = 0.0;
  __syncthreads();
  double va[PF], vb[PF];
  auto fetch = [&](int q) {
    const int64_t base = (int64_t)q * r2;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = tid + u * 256;
      va[u] = ld_ok(Xaa, base + e, e < r2);
      vb[u] = ld_ok(Xab, base + e, e < r2);
    }
  };
  auto deposit = [&]() {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = tid + u * 256;
      if (e < r2) {
        const int row = e / r, col = e - (e / r) * r;
        SA[row * rp + col] = va[u];
        SB[row * rp + col] = vb[u];
      }
    }
  };
  int q = blockIdx.x;
  fetch(q);
  deposit();
  __syncthreads();
  for (;;) {
    const int qn = q + (int)gridDim.x;
    const bool more = qn < nslab;
    if (more) fetch(qn);
    const int k = q / r, p = q - (q / r) * r;
    if (fpart && tid < r) {
      // f partial of the slab: sum_r (X_aa[k,p,r,s] - X_ab[k,p,s,r]) g[p,r], s = tid
      double a = 0.0;
      for (int rr = 0; rr < r; ++rr) a += (SA[rr * rp + tid] - SB[tid * rp + rr]) * g[p * r + rr];
      fpart[(int64_t)q * r + tid] = a;  // [k][p][s]
    }
    // accumulator item v of lane l: output row 16 wave + l/16 + 4v, column 16 cb + l%16
    auto store = [&](const mode_d4 *acc, O &out) {
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int sc = cb * 16 + lr;
        if (sc < r) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = wave * 16 + lk + 4 * v;
            if (i < r) out.put(((int64_t)k * r + i) * ld + (int64_t)p * r + sc, acc[cb][v]);
          }
        }
      }
    };
    {  // L+ and L- (two passes over the slab keep fewer accumulators live)
      mode_d4 ap[CB], am[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        ap[cb] = mode_d4{0.0, 0.0, 0.0, 0.0};
        am[cb] = ap[cb];
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kr = ks * 4 + lk;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          const double xa = SA[kr * rp + cb * 16 + lr], xb = SB[kr * rp + cb * 16 + lr];
          ap[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[ks], xa + xb, ap[cb], 0, 0, 0);
          am[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[ks], xa - xb, am[cb], 0, 0, 0);
        }
      }
      store(ap, Lp);
      store(am, Lm);
    }
    {  // L3
      mode_d4 a3[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) a3[cb] = mode_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kr = ks * 4 + lk;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          a3[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[ks], SB[(cb * 16 + lr) * rp + kr], a3[cb], 0, 0, 0);
      }
      store(a3, L3);
    }
    if (p == r - 1) {
      const int pad = ld - r2;
      for (int e = tid; e < r * pad; e += 256) {
        const int i = e / pad, c = e - (e / pad) * pad;
        const int64_t o = ((int64_t)k * r + i) * ld + r2 + c;
        Lp.put(o, 0.0);
        Lm.put(o, 0.0);
        L3.put(o, 0.0);
      }
    }
    if (!more) break;
    __syncthreads();  // every wave is done with the staged slab
    deposit();
    __syncthreads();
    q = qn;
  }
}

// ---------------------------------------------------------------------------
// G2 tensors (fold of the f and H terms) and the packed pp B operands:
//   G2_aa[k,l,r,s] = H_aa[k,l,r,s] - H_aa[l,k,r,s]
//                    + f[k,r] d_ls - f[k,s] d_lr - f[l,r] d_ks + f[l,s] d_kr
//   G2_ab[k,l,r,s] = H_ab[k,l,r,s] + H_ab[l,k,s,r] + f[k,r] d_ls + f[l,s] d_kr
//   B = A - G2 per block (FP64); G2 kept in FP64 (natural layout).
// Operand rows (k,l), K packed to match the D operands:
//   B_aa[(k,l), (r<s)] = B_aa[k,l,r,s] - B_aa[k,l,s,r]
//   B_S [(k,l), (r<=s)] = B_ab[k,l,r,s] + B_ab[k,l,s,r]
//   B_A [(k,l), (r<s)] = B_ab[k,l,r,s] - B_ab[k,l,s,r]
// One block per row (k,l): the natural B rows are staged in LDS.
// ---------------------------------------------------------------------------
// MIR: the mirrored H_ab row (l,k) is first copied to LDS so that its
// transposed read H_ab[l,k,s,r] is an LDS read, not a stride-r global gather
// (three r x (r+1) LDS arrays instead of two).  LDS rows have stride r + 1 so
// the transposed reads are conflict-free.  The element loops issue the global
// loads of kG2U iterations before using any (a block holds one row, so its
// loads would otherwise wait one latency per iteration).
constexpr int kG2U = 4;

// G2 values of element (rr, s) of row (k, l) from H_aa[k,l,rr,s] (hn),
// H_aa[l,k,rr,s] (hm), H_ab[k,l,rr,s] (bn), H_ab[l,k,s,rr] (bt) and the rows
// fk = f[k,:], fl = f[l,:].
__device__ inline void g2_element(int k, int l, int rr, int s, double hn, double hm, double bn, double bt,
                                  const double *fk, const double *fl, double &gaa, double &gab) {
  gaa = hn - hm;
  if (l == s) gaa += fk[rr];
  if (l == rr) gaa -= fk[s];
  if (k == s) gaa -= fl[rr];
  if (k == rr) gaa += fl[s];
  gab = bn + bt;
  if (l == s) gab += fk[rr];
  if (k == rr) gab += fl[s];
}

// Pair tables in LDS: tle[q] = (a << 8) | b for the pairs a <= b in packed
// order, tlt[q] likewise for a < b (r <= 256), so the packing loops do not
// solve for (a, b) per element.
__device__ inline void pair_tables(int r, uint16_t *tle, uint16_t *tlt, int tid, int nt) {
  const int nle = npair_le(r), nlt = npair_lt(r);
  for (int q = tid; q < nle; q += nt) {
    int a, b;
    unpair_le(r, q, a, b);
    tle[q] = (uint16_t)((a << 8) | b);
  }
  for (int q = tid; q < nlt; q += nt) {
    int a, b;
    unpair_lt(r, q, a, b);
    tlt[q] = (uint16_t)((a << 8) | b);
  }
}

// Packed pp B operand row `row` (K padding included) from the natural rows
// B_aa = ba, B_ab = bb held in LDS with row stride rp; pair tables from
// pair_tables, or null to solve for each pair.
template <class O>
__device__ inline void g2_pack(int r, int64_t row, int ld_lt, int ld_le, const double *ba, const double *bb,
                               int rp, const uint16_t *tle, const uint16_t *tlt, const O &Baa, const O &BS,
                               const O &BA, int tid, int nt) {
  const int nle = npair_le(r), nlt = npair_lt(r);
  for (int q = tid; q < ld_le; q += nt) {
    double v = 0.0;
    if (q < nle) {
      int a, b;
      if (tle) {
        a = tle[q] >> 8;
        b = tle[q] & 255;
      } else {
        unpair_le(r, q, a, b);
      }
      v = bb[a * rp + b] + bb[b * rp + a];
    }
    BS.put(row * ld_le + q, v);
  }
  for (int q = tid; q < ld_lt; q += nt) {
    double va = 0.0, vb = 0.0;
    if (q < nlt) {
      int a, b;
      if (tlt) {
        a = tlt[q] >> 8;
        b = tlt[q] & 255;
      } else {
        unpair_lt(r, q, a, b);
      }
      va = ba[a * rp + b] - ba[b * rp + a];
      vb = bb[a * rp + b] - bb[b * rp + a];
    }
    Baa.put(row * ld_lt + q, va);
    BA.put(row * ld_lt + q, vb);
  }
}

// LDS bytes of the two pair tables of r (rounded to 16)
__host__ __device__ inline size_t pair_table_bytes(int r) {
  return ((size_t)(r * (r + 1) / 2 + r * (r - 1) / 2) * sizeof(uint16_t) + 15) / 16 * 16;
}

template <class O, bool MIR>
__global__ void __launch_bounds__(512)
k_g2(int r, int ld_lt, int ld_le, const double *__restrict__ Aaa, const double *__restrict__ Aab,
     const double *__restrict__ Haa, const double *__restrict__ Hab, const double *__restrict__ f,
     double *__restrict__ G2aa, double *__restrict__ G2ab, O Baa, O BS, O BA, int use_tables) {
  extern __shared__ double g2_smem[];
  constexpr int NT = 512, U = kG2U;
  const int r2 = r * r, RP = r + 1;
  const int row = blockIdx.x;
  const int k = row / r, l = row - (row / r) * r;
  const int64_t nat0 = (int64_t)row * r2, mir0 = ((int64_t)l * r + k) * r2;
  double *ba = g2_smem, *bb = g2_smem + r * RP, *mh = g2_smem + 2 * r * RP;
  uint16_t *tle = nullptr, *tlt = nullptr;
  const int tid = threadIdx.x;
  if (use_tables) {
    tle = reinterpret_cast<uint16_t *>(g2_smem + (MIR ? 3 : 2) * r * RP);
    tlt = tle + npair_le(r);
    pair_tables(r, tle, tlt, tid, NT);
  }
  if constexpr (MIR) {
    for (int base = 0; base < r2; base += NT * U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = base + u * NT + tid;
        v[u] = ld_ok(Hab, mir0 + e, e < r2);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = base + u * NT + tid;
        if (e < r2) {
          const int x = e / r, y = e - (e / r) * r;
          mh[x * RP + y] = v[u];
        }
      }
    }
    __syncthreads();
  }
  for (int base = 0; base < r2; base += NT * U) {
    double hn[U], hm[U], bn[U], bm[U], an[U], aab[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * NT + tid;
      const bool ok = e < r2;
      const int ee = ok ? e : 0;
      const int rr = ee / r, s = ee - (ee / r) * r;
      hn[u] = ld_ok(Haa, nat0 + e, ok);
      hm[u] = ld_ok(Haa, mir0 + e, ok);
      bn[u] = ld_ok(Hab, nat0 + e, ok);
      if constexpr (!MIR) bm[u] = ld_ok(Hab, mir0 + (int64_t)s * r + rr, ok);
      an[u] = ld_ok(Aaa, nat0 + e, ok);
      aab[u] = ld_ok(Aab, nat0 + e, ok);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * NT + tid;
      if (e >= r2) continue;
      const int rr = e / r, s = e - (e / r) * r;
      double gaa, gab;
      g2_element(k, l, rr, s, hn[u], hm[u], bn[u], MIR ? mh[s * RP + rr] : bm[u], f + k * r, f + l * r, gaa,
                 gab);
      G2aa[nat0 + e] = gaa;
      G2ab[nat0 + e] = gab;
      ba[rr * RP + s] = an[u] - gaa;
      bb[rr * RP + s] = aab[u] - gab;
    }
  }
  __syncthreads();
  g2_pack(r, row, ld_lt, ld_le, ba, bb, RP, tle, tlt, Baa, BS, BA, tid, NT);
}

// ---------------------------------------------------------------------------
// G2 fused with C^T = alpha g G2 g (r <= 52): the G2 rows never leave LDS.
// Persistent blocks of 4 waves walk the items (row (k,l), side), side 0 the
// alpha-alpha block and side 1 the alpha-beta block: an item reads three input
// rows (the natural and the mirrored H row, the A row), and a block needs the
// LDS of one side only, so two blocks share a CU and one block's loads and
// stores proceed while the other runs its MFMAs.  Per item: the mirrored H_ab
// row is staged (alpha-beta only); G2 of the side (a zero-padded r x r matrix,
// row stride 4 KS + 2) and B = A - G2 go to LDS; the side's packed pp B
// operand rows are written; then U^T = g G2^T and C = alpha g U on the FP64
// MFMA, with g (symmetric) as the A operand held in registers (wave w: rows
// 16 w ..) and the B operands read transposed from LDS (conflict-free for a
// row stride = 2 mod 4).
// ---------------------------------------------------------------------------
template <class O, int KS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_g2c(int r, int ld_lt, int ld_le, const double *__restrict__ Aaa, const double *__restrict__ Aab,
      const double *__restrict__ Haa, const double *__restrict__ Hab, const double *__restrict__ f,
      const double *__restrict__ g, double alpha, double *__restrict__ Caa, double *__restrict__ Cab,
      O Baa, O BS, O BA, int nitem) {
  constexpr int NT = 256;
  constexpr int NB = (4 * KS + 15) / 16, NR = 16 * NB, RP = 4 * KS + 2;
  static_assert(NB <= 4, "one 16-row block of U per wave");
  constexpr int PF = (4 * KS * 4 * KS + NT - 1) / NT;  // elements of one row per thread (r <= 4 KS)
  extern __shared__ double g2c_smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int r2 = r * r;
  const int zlen = 2 * r * RP > NR * RP ? 2 * r * RP : NR * RP;
  double *const G = g2c_smem;       // [NR][RP] G2 of the item's side
  double *const Z = G + NR * RP;    // B and the mirrored H_ab row ([r][RP] each), later U^T [NR][RP]
  double *const Bs = Z, *const MH = Z + r * RP;
  double *const FK = Z + zlen, *const FL = FK + r;  // rows k and l of f
  uint16_t *const tle = reinterpret_cast<uint16_t *>(FL + r), *const tlt = tle + npair_le(r);
  pair_tables(r, tle, tlt, tid, NT);
  double afr[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int x = wave * 16 + lr, y = ks * 4 + lk;
    const bool ok = x < r && y < r;
    const double v = ld_ok(g, (int64_t)x * r + y, ok);
    afr[ks] = ok ? v : 0.0;
  }
  for (int e = tid; e < NR * RP; e += NT) G[e] = 0.0;
  const int nlt = npair_lt(r), nle = npair_le(r);
  __syncthreads();  // zero fill of G complete
  for (int item = blockIdx.x; item < nitem; item += gridDim.x) {
    const int row = item >> 1, side = item & 1;
    const int k = row / r, l = row - (row / r) * r;
    const int64_t nat0 = (int64_t)row * r2, mir0 = ((int64_t)l * r + k) * r2;
    const double *H = side ? Hab : Haa, *A = side ? Aab : Aaa;
    double vn[PF], vm[PF], va[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = tid + u * NT;
      const bool ok = e < r2;
      vn[u] = ld_ok(H, nat0 + e, ok);
      vm[u] = ld_ok(H, mir0 + e, ok);
      va[u] = ld_ok(A, nat0 + e, ok);
    }
    if (side) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int e = tid + u * NT;
        if (e < r2) {
          const int x = e / r, y = e - (e / r) * r;
          MH[x * RP + y] = vm[u];
        }
      }
    }
    if (tid < r) FK[tid] = f[k * r + tid];
    else if (tid >= 128 && tid - 128 < r) FL[tid - 128] = f[l * r + tid - 128];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int e = tid + u * NT;
      if (e < r2) {
        const int rr = e / r, s = e - (e / r) * r;
        double gaa, gab;
        if (side)
          g2_element(k, l, rr, s, 0.0, 0.0, vn[u], MH[s * RP + rr], FK, FL, gaa, gab);
        else
          g2_element(k, l, rr, s, vn[u], vm[u], 0.0, 0.0, FK, FL, gaa, gab);
        const double v = side ? gab : gaa;
        G[rr * RP + s] = v;
        Bs[rr * RP + s] = va[u] - v;
      }
    }
    __syncthreads();
    // packed pp B operand rows of the side (K padding included)
    if (side) {
      for (int q = tid; q < ld_le; q += NT) {
        double v = 0.0;
        if (q < nle) {
          const int a = tle[q] >> 8, b = tle[q] & 255;
          v = Bs[a * RP + b] + Bs[b * RP + a];
        }
        BS.put((int64_t)row * ld_le + q, v);
      }
    }
    for (int q = tid; q < ld_lt; q += NT) {
      double v = 0.0;
      if (q < nlt) {
        const int a = tlt[q] >> 8, b = tlt[q] & 255;
        v = Bs[a * RP + b] - Bs[b * RP + a];
      }
      (side ? BA : Baa).put((int64_t)row * ld_lt + q, v);
    }
    __syncthreads();  // B and the mirrored row are read; U^T may overwrite them
    mode_d4 acc[NB];
    if (wave < NB) {
      // U^T[j][r'] = sum_s g[j][s] G2[r'][s]; accumulator item v of lane l:
      // row j = 16 wave + l/16 + 4v, column r' = 16 cb + l%16
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) acc[cb] = mode_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kr = ks * 4 + lk;
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[ks], G[(cb * 16 + lr) * RP + kr], acc[cb], 0, 0, 0);
      }
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
        if (cb * 16 + lr < 4 * KS) {
#pragma unroll
          for (int v = 0; v < 4; ++v) Z[(wave * 16 + lk + 4 * v) * RP + cb * 16 + lr] = acc[cb][v];
        }
    }
    __syncthreads();
    if (wave < NB) {
      // C[i][j] = alpha sum_r' g[i][r'] U^T[j][r']
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) acc[cb] = mode_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kr = ks * 4 + lk;
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[ks], Z[(cb * 16 + lr) * RP + kr], acc[cb], 0, 0, 0);
      }
      double *dst = (side ? Cab : Caa) + (int64_t)row * r2;
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const int j = cb * 16 + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = wave * 16 + lk + 4 * v;
          if (i < r && j < r) dst[i * r + j] = alpha * acc[cb][v];
        }
      }
    }
    __syncthreads();  // G and U^T are read before the next item overwrites them
  }
}

// ---------------------------------------------------------------------------
// Assembly of S (before the (ij)<->(kl) exchange), FP64:
//   S_aa = Z_aa - (g_il t_jk - g_jl t_ik - g_ik t_jl + g_jk t_il)
//               - (E1[i,j,k,l] - E1[j,i,k,l] - E1[i,j,l,k] + E1[j,i,l,k])
//   S_ab = Z_ab + g_jl t_ik + g_ik t_jl
//               - (E2[i,j,k,l] + E2[j,i,l,k] - E3[i,j,k,l] - E3[j,i,l,k])
// with E1 = P+ + P-, E2 = P+ - P- (all stored [i,j,k,l]).  The pp products
// come packed: Z_aa = +-Zp_aa[(i<j)] (0 on i = j), and
// Z_ab[i,j] = 1/2 (Z_S[(i<=j)] +- Z_A[(i<j)]) (sign + for i < j).
// One block per unordered pair {i <= j} and chunk of kKC values of k writes
// those rows of the slabs S[i,j,:,:] and S[j,i,:,:]; it stages, for both slabs (i,j)
// and (j,i) of P+, P- and E3, the rows X[.,.,k,:] and the column stripes
// X[.,.,:,k] in LDS, so every global read is a contiguous run.
// ---------------------------------------------------------------------------
constexpr int kKC = 8;

__global__ void __launch_bounds__(256)
k_assemble(int r, const double *__restrict__ g, const double *__restrict__ t,
           const double *__restrict__ Zaa, const double *__restrict__ ZS, const double *__restrict__ ZA,
           const double *__restrict__ Pp, const double *__restrict__ Pm,
           const double *__restrict__ E3, double *__restrict__ Saa, double *__restrict__ Sab) {
  extern __shared__ double asm_smem[];
  // pair index -> (i, j), i <= j
  int i = 0, rem = blockIdx.x;
  while (rem >= r - i) { rem -= r - i; ++i; }
  const int j = i + rem;
  const int64_t r2 = (int64_t)r * r;
  const double *X[3] = {Pp, Pm, E3};
  const int64_t zs0 = (int64_t)blockIdx.x * r2;                        // Z_S row (i<=j)
  const int64_t za0 = i < j ? (int64_t)pair_lt(r, i, j) * r2 : 0;      // Z_aa, Z_A row (i<j)
  const int64_t slab[2] = {((int64_t)i * r + j) * r2, ((int64_t)j * r + i) * r2};
  // rowp[s][x][kk][l] and colp[s][x][l][kk] (padded)
  const int RW = kKC * r, CW = r * (kKC + 1);
  double *rowp = asm_smem;
  double *colp = asm_smem + 6 * RW;
  const int nslab = (i == j) ? 1 : 2;
  {
    const int k0 = blockIdx.y * kKC;
    const int kc = min(kKC, r - k0);
    const int tot = 6 * kc * r;
    for (int base = 0; base < tot; base += 256 * kStage) {
      double vr[kStage], vc[kStage];
      int dr[kStage], dc[kStage];
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int e = base + u * 256 + threadIdx.x;
        const int sx = e / (kc * r), w = e - sx * (kc * r);
        const int s = sx / 3, x = sx - 3 * s;
        const int kk = w / r, l = w - kk * r;      // row stripe X[s][k0+kk][l]
        const int l2 = w / kc, kk2 = w - l2 * kc;  // column stripe X[s][l2][k0+kk2]
        dr[u] = sx * RW + kk * r + l;
        dc[u] = sx * CW + l2 * (kKC + 1) + kk2;
        const bool ok = e < tot;
        const double *Xp = X[ok ? x : 0];
        vr[u] = ld_ok(Xp, slab[ok ? s : 0] + (int64_t)(k0 + kk) * r + l, ok);
        vc[u] = ld_ok(Xp, slab[ok ? s : 0] + (int64_t)l2 * r + k0 + kk2, ok);
      }
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int e = base + u * 256 + threadIdx.x;
        if (e < tot) { rowp[dr[u]] = vr[u]; colp[dc[u]] = vc[u]; }
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nslab * kc * r; e += 256) {
      const int s = e / (kc * r), w = e % (kc * r);
      const int kk = w / r, l = w % r;
      const int k = k0 + kk;
      const int a = s ? j : i, b = s ? i : j;   // output slab (a, b)
      const int o = 1 - s;                      // the other slab (b, a)
      auto R = [&](int sl, int x) { return rowp[(sl * 3 + x) * RW + kk * r + l]; };       // X[sl][k][l]
      auto Cq = [&](int sl, int x) { return colp[(sl * 3 + x) * CW + l * (kKC + 1) + kk]; };  // X[sl][l][k]
      const double e1 = (R(s, 0) + R(s, 1)) - (R(o, 0) + R(o, 1)) - (Cq(s, 0) + Cq(s, 1)) +
                        (Cq(o, 0) + Cq(o, 1));
      const double e2 = (R(s, 0) - R(s, 1)) + (Cq(o, 0) - Cq(o, 1)) - R(s, 2) - Cq(o, 2);
      const double gt_aa = g[a * r + l] * t[b * r + k] - g[b * r + l] * t[a * r + k] -
                           g[a * r + k] * t[b * r + l] + g[b * r + k] * t[a * r + l];
      const double gt_ab = g[b * r + l] * t[a * r + k] + g[a * r + k] * t[b * r + l];
      const int64_t out = slab[s] + (int64_t)k * r + l;
      const int64_t kl = (int64_t)k * r + l;
      const double sg = i == j ? 0.0 : (s ? -1.0 : 1.0);
      const double zaa = sg * Zaa[za0 + kl];
      const double zab = 0.5 * (ZS[zs0 + kl] + sg * ZA[za0 + kl]);
      Saa[out] = zaa - gt_aa - e1;
      Sab[out] = zab + gt_ab - e2;
    }
    __syncthreads();
  }
}

// Whole-slab form of the same assembly (r <= 81), one block per unordered pair
// {i <= j} writing S[i,j,:,:] and S[j,i,:,:].  With E1 = P+ + P- and
// Y = P+ - P- - E3, the ph terms of the two slabs are
//   slab (i,j): e1 = D[k,l] - D[l,k],     e2 = Y[i,j,k,l] + Y[j,i,l,k]
//   slab (j,i): e1 = -(D[k,l] - D[l,k]),  e2 = Y[j,i,k,l] + Y[i,j,l,k]
// with D[k,l] = E1[i,j,k,l] - E1[j,i,k,l].  The block reads the six input
// slabs X[i,j,:,:], X[j,i,:,:] (contiguous r^2 runs, each read once overall),
// keeps D and the two Y slabs in LDS (row stride r + 1, so the transposed
// reads are conflict-free) together with rows i, j of g and t, and writes both
// output slabs in contiguous runs.
constexpr int kAsmThreads = 512;
constexpr int kAsmU = 4;  // loop iterations whose global loads are issued together

__global__ void __launch_bounds__(kAsmThreads)
k_assemble_slab(int r, const double *__restrict__ g, const double *__restrict__ t,
                const double *__restrict__ Zaa, const double *__restrict__ ZS, const double *__restrict__ ZA,
                const double *__restrict__ Pp, const double *__restrict__ Pm,
                const double *__restrict__ E3, double *__restrict__ Saa, double *__restrict__ Sab) {
  extern __shared__ double asm_smem[];
  int i = 0, rem = blockIdx.x;
  while (rem >= r - i) { rem -= r - i; ++i; }
  const int j = i + rem;
  const int r2 = r * r, RP = r + 1, SL = r * RP;
  double *D = asm_smem, *Y0 = asm_smem + SL, *Y1 = asm_smem + 2 * SL;
  double *gi = asm_smem + 3 * SL, *gj = gi + r, *ti = gj + r, *tj = ti + r;
  const int64_t s0 = ((int64_t)i * r + j) * r2, s1 = ((int64_t)j * r + i) * r2;
  constexpr int U = kAsmU;
  const int tid = threadIdx.x;
  for (int base = 0; base < r2; base += kAsmThreads * U) {
    double p0[U], m0[U], x0[U], p1[U], m1[U], x1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * kAsmThreads + tid;
      const bool ok = e < r2;
      p0[u] = ld_ok(Pp, s0 + e, ok); m0[u] = ld_ok(Pm, s0 + e, ok); x0[u] = ld_ok(E3, s0 + e, ok);
      p1[u] = ld_ok(Pp, s1 + e, ok); m1[u] = ld_ok(Pm, s1 + e, ok); x1[u] = ld_ok(E3, s1 + e, ok);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * kAsmThreads + tid;
      if (e >= r2) continue;
      const int k = e / r, l = e - (e / r) * r;
      D[k * RP + l] = (p0[u] + m0[u]) - (p1[u] + m1[u]);
      Y0[k * RP + l] = (p0[u] - m0[u]) - x0[u];
      Y1[k * RP + l] = (p1[u] - m1[u]) - x1[u];
    }
  }
  for (int e = threadIdx.x; e < r; e += kAsmThreads) {
    gi[e] = g[i * r + e]; gj[e] = g[j * r + e];
    ti[e] = t[i * r + e]; tj[e] = t[j * r + e];
  }
  __syncthreads();
  const int64_t zs0 = (int64_t)blockIdx.x * r2;                        // Z_S row (i<=j)
  const int64_t za0 = i < j ? (int64_t)pair_lt(r, i, j) * r2 : 0;      // Z_aa, Z_A row (i<j)
  const bool off = i != j;
  for (int base = 0; base < r2; base += kAsmThreads * U) {
    double vzs[U], vzaa[U], vza[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * kAsmThreads + tid;
      const bool ok = e < r2;
      vzs[u] = ld_ok(ZS, zs0 + e, ok);
      vzaa[u] = ld_ok(Zaa, za0 + e, ok);
      vza[u] = ld_ok(ZA, za0 + e, ok);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * kAsmThreads + tid;
      if (e >= r2) continue;
      const int k = e / r, l = e - (e / r) * r;
      const double zs = vzs[u];
      const double zaa = off ? vzaa[u] : 0.0, za = off ? vza[u] : 0.0;
      const double e1 = D[k * RP + l] - D[l * RP + k];
      // slab (a, b) = (i, j)
      {
        const double gt_aa = gi[l] * tj[k] - gj[l] * ti[k] - gi[k] * tj[l] + gj[k] * ti[l];
        const double gt_ab = gj[l] * ti[k] + gi[k] * tj[l];
        const double e2 = Y0[k * RP + l] + Y1[l * RP + k];
        Saa[s0 + e] = zaa - gt_aa - e1;
        Sab[s0 + e] = 0.5 * (zs + za) + gt_ab - e2;
      }
      if (off) {  // slab (a, b) = (j, i)
        const double gt_aa = gj[l] * ti[k] - gi[l] * tj[k] - gj[k] * ti[l] + gi[k] * tj[l];
        const double gt_ab = gi[l] * tj[k] + gj[k] * ti[l];
        const double e2 = Y1[k * RP + l] + Y0[l * RP + k];
        Saa[s1 + e] = -zaa - gt_aa + e1;
        Sab[s1 + e] = 0.5 * (zs - za) + gt_ab - e2;
      }
    }
  }
}

// Out = S + sigma S^T ((ij)<->(kl)) with S = S' + C^T (C stored [k,l,i,j]),
// on 32 x 32 tiles of the r^2 x r^2 pair matrix.  Out[b,a] = sigma Out[a,b],
// so one block per tile pair (R0 <= C0) reads the (R0, C0) and (C0, R0) tiles
// of S' and C once, writes the (R0, C0) tile and, transposed through LDS, the
// mirrored one.  Optional masked copy (the mask is symmetric under the
// exchange); per-block partial sums of 2 Out_aa^2 + 4 Out_ab^2.
constexpr int kFT = 32;

__global__ void __launch_bounds__(256)
k_finish(int r, double sigma, const double *__restrict__ Saa, const double *__restrict__ Sab,
         const double *__restrict__ Caa, const double *__restrict__ Cab,
         double *__restrict__ Oaa, double *__restrict__ Oab, ActiveBits active,
         double *__restrict__ Maa, double *__restrict__ Mab, double *__restrict__ partial) {
  __shared__ double sA[kFT][kFT + 1], cA[kFT][kFT + 1], sB[kFT][kFT + 1], cB[kFT][kFT + 1];
  __shared__ double red[256];
  const int64_t r2 = (int64_t)r * r;
  const int nt = (int)((r2 + kFT - 1) / kFT);
  int tr, tc;
  unpair_le(nt, blockIdx.x, tr, tc);
  const int64_t R0 = (int64_t)tr * kFT, C0 = (int64_t)tc * kFT;
  const bool diag = tr == tc;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  auto act = [&](int q2) { return (active.w[q2 >> 6] >> (q2 & 63)) & 1ull; };
  auto masked = [&](int64_t row, int64_t col) {
    const int i = (int)(row / r), j = (int)(row % r), k = (int)(col / r), l = (int)(col % r);
    return act(i) && act(j) && act(k) && act(l);
  };
  double acc = 0.0;
  for (int blk = 0; blk < 2; ++blk) {
    const double *S = blk ? Sab : Saa;
    const double *C = blk ? Cab : Caa;
    double *O = blk ? Oab : Oaa;
    double *M = blk ? Mab : Maa;
    const double w = blk ? 4.0 : 2.0;
#pragma unroll
    for (int q = 0; q < kFT; q += 8) {
      const int y = ty + q;
      const int64_t ra = R0 + y, ca = C0 + tx;   // (row, col) tile
      const int64_t rb = C0 + y, cb = R0 + tx;   // mirrored tile
      const bool oka = ra < r2 && ca < r2, okb = rb < r2 && cb < r2;
      const double s1 = ld_ok(S, ra * r2 + ca, oka), c1 = ld_ok(C, ra * r2 + ca, oka);
      const double s2 = ld_ok(S, rb * r2 + cb, okb), c2 = ld_ok(C, rb * r2 + cb, okb);
      sA[y][tx] = oka ? s1 : 0.0;
      cA[y][tx] = oka ? c1 : 0.0;
      sB[y][tx] = okb ? s2 : 0.0;
      cB[y][tx] = okb ? c2 : 0.0;
    }
    __syncthreads();
    // the (R0, C0) tile: v = S[a,b] + C[b,a] + sigma (S[b,a] + C[a,b]); kept in sA
    double v[kFT / 8];
#pragma unroll
    for (int q = 0; q < kFT; q += 8) {
      const int y = ty + q;
      v[q / 8] = (sA[y][tx] + cB[tx][y]) + sigma * (sB[tx][y] + cA[y][tx]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kFT; q += 8) {
      const int y = ty + q;
      sA[y][tx] = v[q / 8];
      const int64_t row = R0 + y, col = C0 + tx;
      if (row < r2 && col < r2) {
        const int64_t e = row * r2 + col;
        O[e] = v[q / 8];
        acc += (diag ? 1.0 : 2.0) * w * v[q / 8] * v[q / 8];
        if (M) M[e] = masked(row, col) ? 0.0 : v[q / 8];
      }
    }
    __syncthreads();
    if (!diag) {
#pragma unroll
      for (int q = 0; q < kFT; q += 8) {
        const int y = ty + q;
        const int64_t row = C0 + y, col = R0 + tx;
        if (row < r2 && col < r2) {
          const double u = sigma * sA[tx][y];
          const int64_t e = row * r2 + col;
          O[e] = u;
          if (M) M[e] = masked(row, col) ? 0.0 : u;
        }
      }
    }
    __syncthreads();
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w2 = 128; w2 > 0; w2 >>= 1) {
    if (threadIdx.x < w2) red[threadIdx.x] += red[threadIdx.x + w2];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Sum of n partials in a fixed order by one block; writes out[0].
__global__ void __launch_bounds__(256)
k_reduce_sum(int64_t n, const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double red[256];
  // eight independent partial sums per thread keep eight loads in flight
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t q = threadIdx.x;
  for (; q + 7 * 256 < n; q += 8 * 256) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += part[q + u * 256];
  }
  for (; q < n; q += 256) a[0] += part[q];
  const double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// Input symmetry check: per block, the largest |x[e] - sign x[perm(e)]| over
// the generators of the symmetry, and the largest |x[e]| (a NaN propagates
// into both).  kind 0: r x r matrix, x[i,j] = x[j,i]; 1: (pq|rs), invariant
// under p<->q, r<->s and (pq)<->(rs); 2: alpha-alpha 2-RDM, antisymmetric
// under i<->j and k<->l, invariant under (ij)<->(kl); 3: alpha-beta 2-RDM,
// invariant under (ij)<->(kl) and (ij)(kl) -> (ji)(lk).
// ---------------------------------------------------------------------------
__device__ inline double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

__global__ void __launch_bounds__(256)
k_sym_check(int r, int kind, const double *__restrict__ x, double *__restrict__ part) {
  __shared__ double rv[256], rm[256];
  const int64_t r2 = (int64_t)r * r;
  const int64_t n = kind == 0 ? r2 : r2 * r2;
  double viol = 0.0, mag = 0.0;
  auto at = [&](int64_t a, int64_t b, int64_t c, int64_t d) { return x[((a * r + b) * r + c) * r + d]; };
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const double v = x[e];
    mag = nan_max(mag, fabs(v));
    if (kind == 0) {
      const int64_t i = e / r, j = e % r;
      viol = nan_max(viol, fabs(v - x[j * r + i]));
      continue;
    }
    const int64_t l = e % r, kk = (e / r) % r, j = (e / r2) % r, i = e / (r2 * r);
    const double sw = at(j, i, kk, l), sk = at(i, j, l, kk), ex = at(kk, l, i, j);
    if (kind == 1) {
      viol = nan_max(viol, fabs(v - sw));
      viol = nan_max(viol, fabs(v - sk));
      viol = nan_max(viol, fabs(v - ex));
    } else if (kind == 2) {
      viol = nan_max(viol, fabs(v + sw));
      viol = nan_max(viol, fabs(v + sk));
      viol = nan_max(viol, fabs(v - ex));
    } else {
      viol = nan_max(viol, fabs(v - ex));
      viol = nan_max(viol, fabs(v - at(j, i, l, kk)));
    }
  }
  rv[threadIdx.x] = viol;
  rm[threadIdx.x] = mag;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rv[threadIdx.x] = nan_max(rv[threadIdx.x], rv[threadIdx.x + w]);
      rm[threadIdx.x] = nan_max(rm[threadIdx.x], rm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rv[0];
    part[2 * blockIdx.x + 1] = rm[0];
  }
}

__global__ void __launch_bounds__(256)
k_sym_reduce(int nb, const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double rv[256], rm[256];
  double viol = 0.0, mag = 0.0;
  for (int q = threadIdx.x; q < nb; q += 256) {
    viol = nan_max(viol, part[2 * q]);
    mag = nan_max(mag, part[2 * q + 1]);
  }
  rv[threadIdx.x] = viol;
  rm[threadIdx.x] = mag;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rv[threadIdx.x] = nan_max(rv[threadIdx.x], rv[threadIdx.x + w]);
      rm[threadIdx.x] = nan_max(rm[threadIdx.x], rm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = rv[0];
    out[1] = rm[0];
  }
}

// ---------------------------------------------------------------------------
// Gram products  out[j,k] = sum_x (w1 P1[j,x] Q1[k,x] + w2 P2[j,x] Q2[k,x]),
// x in [0, r^3) (for t: P = W, Q = A, weights 1 and 2).  A K-split over
// kTBlocks blocks, each reducing its x range into an r x r partial on the FP64
// MFMA: x slabs of kTChunk are staged row-wise in LDS (rows j >= r zero, the
// weights folded into the P rows) and wave w owns the 16-row output blocks
// NBW w ... NBW w + NBW - 1 against every 16-column block.
// ---------------------------------------------------------------------------
constexpr int kTChunk = 32;
constexpr int kTBlocks = 512;
constexpr int kTLdx = kTChunk + 1;  // odd LDS row stride

// NB = ceil(r / 16) output blocks per side (compile time, so the MFMA chains
// are straight-line code); wave w owns block rows w and w + 4.
template <int NB, bool TWO>
__global__ void __launch_bounds__(256)
k_t_partial(int r, const double *__restrict__ P1, const double *__restrict__ Q1,
            const double *__restrict__ P2, const double *__restrict__ Q2, double w1, double w2,
            double *__restrict__ part) {
  extern __shared__ double t_smem[];
  constexpr int rows = NB * 16;
  constexpr int NBW = NB > 4 ? 2 : 1;
  double *sP1 = t_smem, *sQ1 = sP1 + rows * kTLdx, *sP2 = sQ1 + rows * kTLdx, *sQ2 = sP2 + rows * kTLdx;
  const int64_t X = (int64_t)r * r * r;
  const int64_t per = (X + gridDim.x - 1) / gridDim.x;
  const int64_t x0 = (int64_t)blockIdx.x * per, x1 = min(X, x0 + per);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[NBW][NB];
#pragma unroll
  for (int a = 0; a < NBW; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  // The chunk's elements go through registers: the loads of chunk c + 1 are
  // in flight while the MFMAs of chunk c run.
  constexpr int PER = rows * kTChunk / 256;  // elements per thread per array
  static_assert(PER * 256 == rows * kTChunk, "chunk must split evenly over the block");
  double v[PER][4];
  auto fetch = [&](int64_t xc) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = u * 256 + tid;
      const int j = e / kTChunk, c = e - (e / kTChunk) * kTChunk;
      const bool ok = j < r && xc + c < x1;
      const int64_t o = (int64_t)j * X + xc + c;
      v[u][0] = ld_ok(P1, o, ok);
      v[u][1] = ld_ok(Q1, o, ok);
      if constexpr (TWO) {
        v[u][2] = ld_ok(P2, o, ok);
        v[u][3] = ld_ok(Q2, o, ok);
      }
    }
  };
  // (out-of-range elements are zeroed here, not in fetch, so that nothing
  // waits for the loads before the MFMAs)
  auto deposit = [&](int64_t xc) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = u * 256 + tid;
      const int j = e / kTChunk, c = e - (e / kTChunk) * kTChunk;
      const bool ok = j < r && xc + c < x1;
      sP1[j * kTLdx + c] = ok ? w1 * v[u][0] : 0.0;
      sQ1[j * kTLdx + c] = ok ? v[u][1] : 0.0;
      if constexpr (TWO) {
        sP2[j * kTLdx + c] = ok ? w2 * v[u][2] : 0.0;
        sQ2[j * kTLdx + c] = ok ? v[u][3] : 0.0;
      }
    }
  };
  if (x0 < x1) fetch(x0);
  for (int64_t xc = x0; xc < x1; xc += kTChunk) {
    deposit(xc);
    __syncthreads();
    if (xc + kTChunk < x1) fetch(xc + kTChunk);
    if (wave < NB) {
#pragma unroll
      for (int st = 0; st < kTChunk / 4; ++st) {
        const int col = st * 4 + lk;
        double b1[NB], b2[NB];
#pragma unroll
        for (int kb = 0; kb < NB; ++kb) {
          b1[kb] = sQ1[(kb * 16 + lr) * kTLdx + col];
          if constexpr (TWO) b2[kb] = sQ2[(kb * 16 + lr) * kTLdx + col];
        }
#pragma unroll
        for (int a = 0; a < NBW; ++a) {
          // NBW = 2 only for NB > 4: the second row block of wave w is w + 4 (< NB when w < NB - 4)
          const int jb = wave + 4 * a < NB ? wave + 4 * a : wave;
          const double a1 = sP1[(jb * 16 + lr) * kTLdx + col];
#pragma unroll
          for (int kb = 0; kb < NB; ++kb)
            acc[a][kb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1[kb], acc[a][kb], 0, 0, 0);
          if constexpr (TWO) {
            const double a2 = sP2[(jb * 16 + lr) * kTLdx + col];
#pragma unroll
            for (int kb = 0; kb < NB; ++kb)
              acc[a][kb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b2[kb], acc[a][kb], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();  // every wave is done with the chunk before the next deposit
  }
  // accumulator item v of lane l: row lk + 4v, column lr of the 16 x 16 block
  if (wave >= NB) return;
  double *out = part + (int64_t)blockIdx.x * r * r;
#pragma unroll
  for (int a = 0; a < NBW; ++a) {
    if (wave + 4 * a >= NB) break;
    const int jb = wave + 4 * a;
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
      const int k = kb * 16 + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = jb * 16 + lk + 4 * v;
        if (j < r && k < r) out[j * r + k] = acc[a][kb][v];
      }
    }
  }
}

// t[j,k] = sum over the per-block partials of k_t_partial: one wavefront per
// output, lanes stride over the partials, then a shuffle reduction (fixed order).
__global__ void __launch_bounds__(256)
k_t_reduce(int r, int nparts, const double *__restrict__ part, double *__restrict__ t, int accumulate) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= r * r) return;
  double acc = 0.0;
  for (int q = lane; q < nparts; q += 64) acc += part[(int64_t)q * r * r + e];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) t[e] = accumulate ? t[e] + acc : acc;
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

// gamma[p,r] = 2/(N-1) sum_q (d2aa[p,q,r,q] + d2ab[p,q,r,q]): one wavefront per
// output, lanes over q, fixed-order shuffle reduction.
__global__ void __launch_bounds__(256)
k_contract_1rdm(int r, double two_over_nm1, const double *__restrict__ d2aa,
                const double *__restrict__ d2ab, double *__restrict__ g) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= r * r) return;
  const int p = e / r, rr = e % r;
  const int64_t r2 = (int64_t)r * r;
  double acc = 0.0;
  for (int q = lane; q < r; q += 64) {
    const int64_t o = ((int64_t)p * r + q) * r2 + (int64_t)rr * r + q;
    acc += d2aa[o] + d2ab[o];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) g[e] = two_over_nm1 * acc;
}

// Fused step tail (one block computes the traces, one pass updates):
//   traces[0..3] = (Tr d2aa, Tr d2ab, Tr(d2aa + eps U_aa), Tr(d2ab + eps U_ab)),
//   d2 <- (d2 + eps U) * (Tr_in / Tr_new) per block, in place, and the energy
//   partials 2 K_s (d2aa + d2ab) of the updated blocks.  The updated element is
//   fma(eps, U, d2) in both kernels, so the trace matches the update exactly.
// Traces of 2D and of 2D + eps U per block (diagonal elements (p,q,p,q), one
// per thread and 256 per block): partials part[4 b + k], k = Tr d2aa, Tr d2ab,
// Tr (d2aa + eps U_aa), Tr (d2ab + eps U_ab); then summed in block order.
__global__ void __launch_bounds__(256)
k_step_traces(int r, double eps, const double *__restrict__ d2aa, const double *__restrict__ d2ab,
              const double *__restrict__ Uaa, const double *__restrict__ Uab,
              double *__restrict__ part) {
  __shared__ double red[4][256];
  const int64_t r2 = (int64_t)r * r;
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double a = 0.0, b = 0.0, na = 0.0, nb = 0.0;
  if (q < r2) {
    const int64_t d = q * r2 + q;  // element (p,q,p,q) at row = col = p*r+q
    a = d2aa[d];
    b = d2ab[d];
    na = fma(eps, Uaa[d], a);
    nb = fma(eps, Uab[d], b);
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = na;
  red[3][threadIdx.x] = nb;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_step_traces_sum(int nblk, const double *__restrict__ part, double *__restrict__ traces) {
  const int k = threadIdx.x;
  if (k >= 4) return;
  double t = 0.0;
  for (int b = 0; b < nblk; ++b) t += part[4 * b + k];
  traces[k] = t;
}

__global__ void __launch_bounds__(256)
k_step_update(int r, double eps, double inv_nm1, const double *__restrict__ traces,
              const double *__restrict__ h, const double *__restrict__ V,
              const double *__restrict__ Uaa, const double *__restrict__ Uab,
              double *__restrict__ d2aa, double *__restrict__ d2ab, double *__restrict__ partial) {
  __shared__ double red[256];
  const int64_t r2 = (int64_t)r * r;
  const int64_t n4 = r2 * r2;
  const int64_t e = gtid();
  double acc = 0.0;
  if (e < n4) {
    const double sa = traces[0] / traces[2], sb = traces[1] / traces[3];
    const double naa = fma(eps, Uaa[e], d2aa[e]) * sa;
    const double nab = fma(eps, Uab[e], d2ab[e]) * sb;
    d2aa[e] = naa;
    d2ab[e] = nab;
    const int s = e % r, rr = (e / r) % r, q = (e / r2) % r, p = e / (r2 * r);
    double ks = V[(int64_t)p * r2 * r + (int64_t)rr * r2 + (int64_t)q * r + s];
    if (q == s) ks += h[p * r + rr] * inv_nm1;
    if (p == rr) ks += h[q * r + s] * inv_nm1;
    acc = 2.0 * ks * (naa + nab);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_fill(int64_t n, double v, double *__restrict__ p) {
  const int64_t e = gtid();
  if (e < n) p[e] = v;
}

// oa = ca a, ob = cb b over n elements.
__global__ void k_scale2(int64_t n, double ca, const double *__restrict__ a, double cb,
                         const double *__restrict__ b, double *__restrict__ oa, double *__restrict__ ob) {
  const int64_t e = gtid();
  if (e >= n) return;
  oa[e] = ca * a[e];
  ob[e] = cb * b[e];
}

// Partial sums of a[e] b[e]: block q takes the grid-strided elements of its
// threads and leaves one partial in part[q] (fixed order: deterministic).
__global__ void __launch_bounds__(256)
k_dot_partial(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
              double *__restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    acc = fma(a[e], b[e], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
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
  const size_t lds = ((size_t)2 * r * (r + 1) + 2 * (size_t)r) * sizeof(double);
  ACSE_DISPATCH_OUT(prec, {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_w_ph<O>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_w_ph<O>), dim3((unsigned)(r * r)), dim3(256), lds, s, r, ld, g, d2aa, d2ab,
                       make_out<O>(Rp), make_out<O>(Rm), make_out<O>(R3));
  });
  return hipGetLastError();
}

hipError_t launch_d_operand(GemmPrec prec, int r, const double *d2aa, const double *d2ab,
                            const OperandRef &Daa, const OperandRef &DS, const OperandRef &DA,
                            hipStream_t s) {
  const size_t lds = (size_t)2 * r * r * sizeof(double);
  const int ld_lt = (int)ld_pair_lt(r), ld_le = (int)ld_pair_le(r);
  ACSE_DISPATCH_OUT(prec, {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_d_operand<O>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_d_operand<O>), dim3((unsigned)npair_le(r)), dim3(256), lds, s, r, ld_lt, ld_le,
                       d2aa, d2ab, make_out<O>(Daa), make_out<O>(DS), make_out<O>(DA));
  });
  return hipGetLastError();
}

hipError_t launch_zero_kpad(GemmPrec prec, int r, int ld, const OperandRef &o, hipStream_t s) {
  const int64_t n = (int64_t)r * r * (ld - (int64_t)r * r);
  if (n <= 0) return hipSuccess;
  ACSE_DISPATCH_OUT(prec, hipLaunchKernelGGL((k_zero_kpad<O>), grid_for(n), dim3(256), 0, s, r, ld,
                                             make_out<O>(o)));
  return hipGetLastError();
}

template <class O, int KS>
static hipError_t launch_lops_t(int r, int ld, const double *g, const double *Xaa, const double *Xab,
                                O Lp, O Lm, O L3, double *fpart, hipStream_t s) {
  static int resident = 0;  // blocks the device holds at once
  constexpr int NR = ((4 * KS + 15) / 16) * 16;
  const int rp = lops_rp(KS);
  const size_t lds = (size_t)2 * NR * rp * sizeof(double);
  const void *fn = reinterpret_cast<const void *>(&k_lops<O, KS>);
  if (resident == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds);
    if (e != hipSuccess) return e;
    resident = cus * std::max(per_cu, 1);
  }
  const int nslab = r * r;
  hipLaunchKernelGGL((k_lops<O, KS>), dim3(std::min(nslab, resident)), dim3(256), lds, s, r, ld, rp, g, Xaa,
                     Xab, Lp, Lm, L3, nslab, fpart);
  return hipGetLastError();
}

template <class O>
static hipError_t launch_lops_o(int r, int ld, const double *g, const double *Xaa, const double *Xab, O Lp,
                                O Lm, O L3, double *fpart, hipStream_t s) {
  switch ((r + 3) / 4) {
#define ACSE_LOPS(K) \
    case K: return launch_lops_t<O, K>(r, ld, g, Xaa, Xab, Lp, Lm, L3, fpart, s);
    ACSE_LOPS(1) ACSE_LOPS(2) ACSE_LOPS(3) ACSE_LOPS(4) ACSE_LOPS(5) ACSE_LOPS(6) ACSE_LOPS(7)
    ACSE_LOPS(8) ACSE_LOPS(9) ACSE_LOPS(10) ACSE_LOPS(11) ACSE_LOPS(12) ACSE_LOPS(13) ACSE_LOPS(14)
#undef ACSE_LOPS
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_lops(GemmPrec prec, int r, int ld, const double *g, const double *Xaa, const double *Xab,
                       const OperandRef &Lp, const OperandRef &Lm, const OperandRef &L3, double *fpart,
                       hipStream_t s) {
  if (r < 2 || r > kLopsMaxR) return hipErrorInvalidValue;
  ACSE_DISPATCH_OUT(prec, return launch_lops_o(r, ld, g, Xaa, Xab, make_out<O>(Lp), make_out<O>(Lm),
                                               make_out<O>(L3), fpart, s));
  return hipSuccess;
}

hipError_t launch_sym_check(int r, int kind, const double *x, double *part, double *out2, hipStream_t s) {
  constexpr int kNb = 1024;  // 2 kNb partial doubles
  hipLaunchKernelGGL(k_sym_check, dim3(kNb), dim3(256), 0, s, r, kind, x, part);
  hipLaunchKernelGGL(k_sym_reduce, dim3(1), dim3(256), 0, s, kNb, part, out2);
  return hipGetLastError();
}

hipError_t launch_f_reduce(int r, const double *part, double *f, hipStream_t s) {
  hipLaunchKernelGGL(k_f_reduce, dim3((unsigned)((r * r + 3) / 4)), dim3(256), 0, s, r, part, f);
  return hipGetLastError();
}

hipError_t launch_f(int r, const double *Aaa, const double *Aab, const double *g, double *part,
                    double *f, hipStream_t s) {
  const int64_t r3 = (int64_t)r * r * r;
  hipLaunchKernelGGL(k_f_partial, grid_for(r3), dim3(256), 0, s, r, Aaa, Aab, g, part);
  hipLaunchKernelGGL(k_f_reduce, dim3((unsigned)((r * r + 3) / 4)), dim3(256), 0, s, r, part, f);
  return hipGetLastError();
}

// r <= 64: one 16-row block of M per wave, 32-column panels; r <= 96: two
// row blocks per wave, 16-column panels (the prefetch stays at 8 per thread).
// K steps: exact for r <= 64; rounded up to a multiple of 4 above.
// (The wide shape is also selectable at small r, to verify it there.)
template <class O, int COLS, int NRB, bool HAS2, int KS>
static hipError_t launch_mode_t(const ModeArgs &m, O out, hipStream_t s) {
  static int resident[kModeMaxR + 1] = {};  // blocks the device holds at once, by r
  static_assert((size_t)COLS * 4 * KS <= (size_t)ModeShape<COLS>::PF * 256, "panel must fit the prefetch");
  const size_t lds = (size_t)2 * 4 * KS * (COLS + 1) * sizeof(double);  // two panels
  int &res = resident[m.r];
  if (res == 0) {
    const void *fn = reinterpret_cast<const void *>(&k_mode<O, COLS, NRB, HAS2, KS>);
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds);
    if (e != hipSuccess) return e;
    res = cus * std::max(per_cu, 1);
  }
  const int64_t ncols = m.A * m.Bn;
  const int npanels = (int)((ncols + COLS - 1) / COLS);
  if (npanels == 0) return hipSuccess;
  hipLaunchKernelGGL((k_mode<O, COLS, NRB, HAS2, KS>), dim3(std::min(npanels, res)), dim3(256), lds, s,
                     m, out, npanels);
  return hipGetLastError();
}

template <class O, bool HAS2>
static hipError_t launch_mode_h(const ModeArgs &m, O out, hipStream_t s) {
  if (m.wide || m.r > 64)
    return m.r <= 80 ? launch_mode_t<O, 16, 2, HAS2, 20>(m, out, s) : launch_mode_t<O, 16, 2, HAS2, 24>(m, out, s);
  switch ((m.r + 3) / 4) {
#define ACSE_MODE_KS(K) \
    case K: return launch_mode_t<O, 32, 1, HAS2, K>(m, out, s);
    ACSE_MODE_KS(1) ACSE_MODE_KS(2) ACSE_MODE_KS(3) ACSE_MODE_KS(4) ACSE_MODE_KS(5) ACSE_MODE_KS(6)
    ACSE_MODE_KS(7) ACSE_MODE_KS(8) ACSE_MODE_KS(9) ACSE_MODE_KS(10) ACSE_MODE_KS(11)
    ACSE_MODE_KS(12) ACSE_MODE_KS(13) ACSE_MODE_KS(14) ACSE_MODE_KS(15) ACSE_MODE_KS(16)
#undef ACSE_MODE_KS
    default: return hipErrorInvalidValue;
  }
}

template <class O>
static hipError_t launch_mode_o(const ModeArgs &m, O out, hipStream_t s) {
  return m.in2 ? launch_mode_h<O, true>(m, out, s) : launch_mode_h<O, false>(m, out, s);
}

hipError_t launch_mode(GemmPrec prec, const ModeArgs &m, const OperandRef &out, hipStream_t s) {
  if (m.r < 2 || m.r > kModeMaxR) return hipErrorInvalidValue;
  if (m.accumulate) {
    if (prec != GEMM_F64) return hipErrorInvalidValue;
    return launch_mode_o(m, OutF64Acc{static_cast<double *>(out.hi)}, s);
  }
  ACSE_DISPATCH_OUT(prec, return launch_mode_o(m, make_out<O>(out), s));
  return hipSuccess;
}

hipError_t launch_g2(GemmPrec prec, int r, bool general, const double *Aaa, const double *Aab,
                     const double *Haa, const double *Hab, const double *f, double *G2aa, double *G2ab,
                     const OperandRef &Baa, const OperandRef &BS, const OperandRef &BA, hipStream_t s) {
  const size_t lds2 = (size_t)2 * r * (r + 1) * sizeof(double);
  const size_t lds3 = lds2 + (size_t)r * (r + 1) * sizeof(double);
  const bool mir = !general && lds3 <= kMaxLds;
  const int tables = !general && (mir ? lds3 : lds2) + pair_table_bytes(r) <= kMaxLds;
  const size_t lds = (mir ? lds3 : lds2) + (tables ? pair_table_bytes(r) : 0);
  const int ld_lt = (int)ld_pair_lt(r), ld_le = (int)ld_pair_le(r);
  auto go = [&](auto kern, auto tag) -> hipError_t {
    using O = decltype(tag);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)(r * r)), dim3(512), lds, s, r, ld_lt, ld_le, Aaa, Aab, Haa,
                       Hab, f, G2aa, G2ab, make_out<O>(Baa), make_out<O>(BS), make_out<O>(BA), tables);
    return hipGetLastError();
  };
  if (prec == GEMM_F64)
    return mir ? go(k_g2<OutF64, true>, OutF64{}) : go(k_g2<OutF64, false>, OutF64{});
  if (prec == GEMM_F32)
    return mir ? go(k_g2<OutF32, true>, OutF32{}) : go(k_g2<OutF32, false>, OutF32{});
  return mir ? go(k_g2<OutBF16x3, true>, OutBF16x3{}) : go(k_g2<OutBF16x3, false>, OutBF16x3{});
}

template <class O, int KS>
static hipError_t launch_g2c_t(int r, const double *Aaa, const double *Aab, const double *Haa, const double *Hab,
                               const double *f, const double *g, double alpha, double *Caa, double *Cab, O Baa,
                               O BS, O BA, hipStream_t s) {
  static int resident[kG2cMaxR + 1] = {};  // blocks the device holds at once, by r
  constexpr int NR = 16 * ((4 * KS + 15) / 16), RP = 4 * KS + 2;
  const size_t lds =
      ((size_t)NR * RP + std::max((size_t)2 * r * RP, (size_t)NR * RP) + 2 * (size_t)r) * sizeof(double) +
      pair_table_bytes(r);
  const void *fn = reinterpret_cast<const void *>(&k_g2c<O, KS>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (resident[r] == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds);
    if (e != hipSuccess) return e;
    resident[r] = cus * std::max(per_cu, 1);
  }
  const int nitem = 2 * r * r;  // (row, side)
  hipLaunchKernelGGL((k_g2c<O, KS>), dim3(std::min(nitem, resident[r])), dim3(256), lds, s, r,
                     (int)ld_pair_lt(r), (int)ld_pair_le(r), Aaa, Aab, Haa, Hab, f, g, alpha, Caa, Cab, Baa, BS,
                     BA, nitem);
  return hipGetLastError();
}

template <class O>
static hipError_t launch_g2c_o(int r, const double *Aaa, const double *Aab, const double *Haa, const double *Hab,
                               const double *f, const double *g, double alpha, double *Caa, double *Cab, O Baa,
                               O BS, O BA, hipStream_t s) {
  switch ((r + 3) / 4) {
#define ACSE_G2C(K) \
    case K: return launch_g2c_t<O, K>(r, Aaa, Aab, Haa, Hab, f, g, alpha, Caa, Cab, Baa, BS, BA, s);
    ACSE_G2C(1) ACSE_G2C(2) ACSE_G2C(3) ACSE_G2C(4) ACSE_G2C(5) ACSE_G2C(6) ACSE_G2C(7) ACSE_G2C(8)
    ACSE_G2C(9) ACSE_G2C(10) ACSE_G2C(11) ACSE_G2C(12) ACSE_G2C(13)
#undef ACSE_G2C
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_g2c(GemmPrec prec, int r, const double *Aaa, const double *Aab, const double *Haa,
                      const double *Hab, const double *f, const double *g, double alpha, double *Caa, double *Cab,
                      const OperandRef &Baa, const OperandRef &BS, const OperandRef &BA, hipStream_t s) {
  if (r < 2 || r > kG2cMaxR) return hipErrorInvalidValue;
  ACSE_DISPATCH_OUT(prec, return launch_g2c_o(r, Aaa, Aab, Haa, Hab, f, g, alpha, Caa, Cab, make_out<O>(Baa),
                                              make_out<O>(BS), make_out<O>(BA), s));
  return hipSuccess;
}

hipError_t launch_assemble(int r, bool general, const double *g, const double *t,
                           const double *Zaa, const double *ZS, const double *ZA, const double *Pp,
                           const double *Pm, const double *E3, double *Saa, double *Sab, hipStream_t s) {
  const unsigned npairs = (unsigned)(r * (r + 1) / 2);
  const size_t slab_lds = ((size_t)3 * r * (r + 1) + 4 * (size_t)r) * sizeof(double);
  if (!general && slab_lds <= kMaxLds) {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_assemble_slab),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)slab_lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_assemble_slab, dim3(npairs), dim3(kAsmThreads), slab_lds, s, r, g, t, Zaa, ZS, ZA,
                       Pp, Pm, E3, Saa, Sab);
    return hipGetLastError();
  }
  const size_t lds = (size_t)6 * (kKC * r + r * (kKC + 1)) * sizeof(double);
  hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_assemble),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_assemble, dim3(npairs, (unsigned)((r + kKC - 1) / kKC)), dim3(256), lds, s, r, g,
                     t, Zaa, ZS, ZA, Pp, Pm, E3, Saa, Sab);
  return hipGetLastError();
}

hipError_t launch_finish(int r, double sigma, const double *Saa, const double *Sab,
                         const double *Caa, const double *Cab, double *Oaa, double *Oab,
                         const ActiveBits &active, double *Maa, double *Mab, double *partial,
                         double *sum_out, hipStream_t s) {
  const int64_t nt = ((int64_t)r * r + kFT - 1) / kFT;
  const int64_t nb = nt * (nt + 1) / 2;
  hipLaunchKernelGGL(k_finish, dim3((unsigned)nb), dim3(256), 0, s, r, sigma, Saa, Sab, Caa, Cab, Oaa,
                     Oab, active, Maa, Mab, partial);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, nb, partial, sum_out);
  return hipGetLastError();
}

int64_t finish_partials(int r) {
  const int64_t nt = ((int64_t)r * r + kFT - 1) / kFT;
  return std::max<int64_t>(nt * nt, ((int64_t)r * r * r * r + 255) / 256);
}

hipError_t launch_t_reduce(int r, int nparts, const double *part, double *t, hipStream_t s,
                           int accumulate) {
  hipLaunchKernelGGL(k_t_reduce, dim3((unsigned)((r * r + 3) / 4)), dim3(256), 0, s, r, nparts, part, t,
                     accumulate);
  return hipGetLastError();
}

int t_partial_blocks() { return kTBlocks; }

template <int NB>
static hipError_t launch_gram_nb(int r, const double *P1, const double *Q1, double w1,
                                 const double *P2, const double *Q2, double w2, double *part,
                                 hipStream_t s) {
  const size_t lds = (size_t)4 * NB * 16 * kTLdx * sizeof(double);
  auto go = [&](auto kern) -> hipError_t {
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3(kTBlocks), dim3(256), lds, s, r, P1, Q1, P2, Q2, w1, w2, part);
    return hipGetLastError();
  };
  return P2 ? go(k_t_partial<NB, true>) : go(k_t_partial<NB, false>);
}

hipError_t launch_gram(int r, const double *P1, const double *Q1, double w1, const double *P2,
                       const double *Q2, double w2, double *part, double *out, int accumulate,
                       hipStream_t s, bool wide) {
  if (!P2) { Q2 = nullptr; w2 = 0.0; }
  hipError_t err;
  switch (wide ? 6 : (r + 15) / 16) {
    case 1: err = launch_gram_nb<1>(r, P1, Q1, w1, P2, Q2, w2, part, s); break;
    case 2: err = launch_gram_nb<2>(r, P1, Q1, w1, P2, Q2, w2, part, s); break;
    case 3: err = launch_gram_nb<3>(r, P1, Q1, w1, P2, Q2, w2, part, s); break;
    case 4: err = launch_gram_nb<4>(r, P1, Q1, w1, P2, Q2, w2, part, s); break;
    case 5: err = launch_gram_nb<5>(r, P1, Q1, w1, P2, Q2, w2, part, s); break;
    default: err = launch_gram_nb<6>(r, P1, Q1, w1, P2, Q2, w2, part, s); break;
  }
  if (err != hipSuccess) return err;
  return launch_t_reduce(r, kTBlocks, part, out, s, accumulate);
}

hipError_t launch_t(int r, const double *Waa, const double *Aaa, const double *Wab,
                    const double *Aab, double *part, double *t, hipStream_t s, bool wide) {
  return launch_gram(r, Waa, Aaa, 1.0, Wab, Aab, 2.0, part, t, 0, s, wide);
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

hipError_t launch_step_tail(int r, int N, double eps, const double *h, const double *V,
                            const double *Uaa, const double *Uab, double *d2aa, double *d2ab,
                            double *traces, double *partial, double *E_out, hipStream_t s) {
  const int64_t n4 = (int64_t)r * r * r * r;
  const int64_t nb = (n4 + 255) / 256;
  // trace partials in `partial` (4 per 256 diagonal elements, at most 144 at
  // r = 96; the buffer holds at least 32 and r^4/256 doubles), then the energy
  // partials of the update
  const int nbt = (int)(((int64_t)r * r + 255) / 256);
  hipLaunchKernelGGL(k_step_traces, dim3((unsigned)nbt), dim3(256), 0, s, r, eps, d2aa, d2ab, Uaa, Uab, partial);
  hipLaunchKernelGGL(k_step_traces_sum, dim3(1), dim3(64), 0, s, nbt, partial, traces);
  hipLaunchKernelGGL(k_step_update, dim3((unsigned)nb), dim3(256), 0, s, r, eps, 1.0 / (N - 1), traces,
                     h, V, Uaa, Uab, d2aa, d2ab, partial);
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
  hipLaunchKernelGGL(k_contract_1rdm, dim3((unsigned)((r * r + 3) / 4)), dim3(256), 0, s, r, 2.0 / (N - 1),
                     d2aa, d2ab, g);
  return hipGetLastError();
}

hipError_t launch_scale2(int64_t n, double ca, const double *a, double cb, const double *b, double *oa,
                         double *ob, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale2, grid_for(n), dim3(256), 0, s, n, ca, a, cb, b, oa, ob);
  return hipGetLastError();
}

hipError_t launch_dot(int64_t n, const double *a, const double *b, double *part, double *out,
                      hipStream_t s) {
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (n + 255) / 256));
  hipLaunchKernelGGL(k_dot_partial, dim3((unsigned)nb), dim3(256), 0, s, n, a, b, part);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(256), 0, s, nb, part, out);
  return hipGetLastError();
}

hipError_t launch_fill(int64_t n, double v, double *p, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, grid_for(n), dim3(256), 0, s, n, v, p);
  return hipGetLastError();
}

}  // namespace acse
