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
// One block per destination row (32-bit index arithmetic within the row).
constexpr int kPermU = 10;

template <class O>
__device__ __forceinline__ void perm_row(const PermArgs &a, const O &out, int row) {
  const int r = a.r, r2 = r * r;
  const int64_t o = (int64_t)row * a.ld;
  const int ld = (int)a.ld;
  if (row >= r2) {
    if (!a.accumulate)
      for (int col = threadIdx.x; col < ld; col += 256) out.put(o + col, 0.0);
    return;
  }
  const int i0 = row / r, i1 = row - (row / r) * r;
  const int64_t b1 = i0 * a.s1[0] + i1 * a.s1[1];
  const int64_t b2 = a.src2 ? i0 * a.s2[0] + i1 * a.s2[1] : 0;
  // the loads of kPermU columns are issued before any is used
  for (int c0 = 0; c0 < ld; c0 += 256 * kPermU) {
    double v1[kPermU], v2[kPermU];
#pragma unroll
    for (int u = 0; u < kPermU; ++u) {
      const int col = c0 + u * 256 + threadIdx.x;
      const bool ok = col < r2;
      const int cc = ok ? col : 0;
      const int i2 = cc / r, i3 = cc - (cc / r) * r;
      v1[u] = a.src1[b1 + i2 * a.s1[2] + i3 * a.s1[3]];
      v2[u] = a.src2 ? a.src2[b2 + i2 * a.s2[2] + i3 * a.s2[3]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPermU; ++u) {
      const int col = c0 + u * 256 + threadIdx.x;
      if (col >= ld) break;
      if (col < r2) out.put(o + col, a.c1 * v1[u] + (a.src2 ? a.c2 * v2[u] : 0.0));
      else if (!a.accumulate) out.put(o + col, 0.0);
    }
  }
}

template <class O>
__global__ void __launch_bounds__(256)
k_permute4(PermArgs a, O out) {
  perm_row(a, out, (int)blockIdx.x);
}

// The same permute when a source's unit-stride index is destination position
// q < 3 (so the elementwise form reads it with a stride): one block per value
// of the two other leading positions moves the r x r slice (position q,
// position 3) through LDS, read with q and written with position 3 as the fast
// index.  Each source is either staged that way or, when its unit stride is
// position 3, read directly in the write loop.  Padding rows and columns are
// left to k_permute4_pad.
struct SliceStrides {
  int64_t s1a, s1b, s1q, s2a, s2b, s2q;  // source strides of fixed positions 1, 2 and of q
  int64_t oq, oa, ob;                    // destination offsets of positions q, fixed 1, fixed 2
  int stage1, stage2;                    // which sources go through LDS
};

template <class O>
__device__ __forceinline__ void perm_slice(const PermArgs &a, const SliceStrides &t, const O &out, int bid,
                                           double *ps_smem) {
  const int r = a.r, rp = r + 1;
  const int x1 = bid / r, x2 = bid - (bid / r) * r;
  const int64_t b1 = x1 * t.s1a + x2 * t.s1b;
  const int64_t b2 = a.src2 ? x1 * t.s2a + x2 * t.s2b : 0;
  const bool two = a.src2 != nullptr;
  const int r2 = r * r;
  for (int e0 = 0; e0 < r2; e0 += 256 * kPermU) {
    double v1[kPermU], v2[kPermU];
#pragma unroll
    for (int u = 0; u < kPermU; ++u) {
      const int e = e0 + u * 256 + threadIdx.x;
      const int ee = e < r2 ? e : 0;
      const int tq = ee % r, t3 = ee / r;  // fast: position q (unit source stride)
      v1[u] = t.stage1 ? a.src1[b1 + tq + t3 * a.s1[3]] : 0.0;
      v2[u] = two && t.stage2 ? a.src2[b2 + tq + t3 * a.s2[3]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPermU; ++u) {
      const int e = e0 + u * 256 + threadIdx.x;
      if (e >= r2) break;
      const int tq = e % r, t3 = e / r;
      ps_smem[t3 * rp + tq] = a.c1 * v1[u] + a.c2 * v2[u];
    }
  }
  __syncthreads();
  const int64_t base = x1 * t.oa + x2 * t.ob;
  for (int e = threadIdx.x; e < r2; e += 256) {
    const int t3 = e % r, tq = e / r;  // fast: position 3 (contiguous destination)
    double v = ps_smem[t3 * rp + tq];
    if (!t.stage1) v += a.c1 * a.src1[b1 + tq * t.s1q + t3];
    if (two && !t.stage2) v += a.c2 * a.src2[b2 + tq * t.s2q + t3];
    out.put(base + tq * t.oq + t3, v);
  }
}

template <class O>
__global__ void __launch_bounds__(256)
k_permute4_slice(PermArgs a, SliceStrides t, O out) {
  extern __shared__ double ps_smem[];
  perm_slice(a, t, out, (int)blockIdx.x, ps_smem);
}

// zero padding of an operand-layout permute destination: rows >= r^2 and the
// columns >= r^2 of the first r^2 rows
template <class O>
__device__ __forceinline__ void perm_pad(const PermArgs &a, const O &out, int64_t e) {
  const int64_t r2 = (int64_t)a.r * a.r;
  const int64_t padc = a.ld - r2;
  const int64_t n1 = r2 * padc;  // column padding of the first r^2 rows
  if (e < n1) {
    out.put((e / padc) * a.ld + r2 + e % padc, 0.0);
  } else if (e - n1 < (a.rows - r2) * a.ld) {
    out.put(r2 * a.ld + (e - n1), 0.0);
  }
}

template <class O>
__global__ void k_permute4_pad(PermArgs a, O out) {
  perm_pad(a, out, vtid());
}

// Up to kMaxPermJobs independent permutes (distinct destinations, no source
// another job writes) in one launch: the blocks of each job's main pass (one
// per destination row, or one per slice), then the padding blocks of the
// slice-form jobs; each block finds its job by the block prefix sums.
template <class O>
struct PermBatch {
  PermArgs a[kMaxPermJobs];
  SliceStrides t[kMaxPermJobs];
  O out[kMaxPermJobs];
  int slice[kMaxPermJobs];
  int start[kMaxPermJobs + 1];   // main blocks of job j: [start[j], start[j+1])
  int pstart[kMaxPermJobs + 1];  // padding blocks, numbered after all main blocks
  int count;
};

static_assert(sizeof(PermBatch<VOutBF16x3>) <= 4096 - 64, "kernel arguments must fit in 4 KiB");

template <class O>
__global__ void __launch_bounds__(256)
k_permute4_batch(PermBatch<O> b) {
  extern __shared__ double ps_smem[];
  const int bid = blockIdx.x;
  const int nmain = b.start[b.count];
  if (bid < nmain) {
    int j = 0;
    while (j + 1 < b.count && bid >= b.start[j + 1]) ++j;
    const int local = bid - b.start[j];
    if (b.slice[j]) perm_slice(b.a[j], b.t[j], b.out[j], local, ps_smem);
    else perm_row(b.a[j], b.out[j], local);
    return;
  }
  const int pb = bid - nmain;
  int j = 0;
  while (j + 1 < b.count && pb >= b.pstart[j + 1]) ++j;
  perm_pad(b.a[j], b.out[j], (int64_t)(pb - b.pstart[j]) * 256 + threadIdx.x);
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

// Slab form of the same contraction, for terms whose output pair takes one
// index from each index pair of T: x = index px in {0, 1} with u the other of
// (0, 1), y = index py in {2, 3} with v the other of (2, 3).  The slab
// S = T_t[i,j,:,:] (rows: index 2) then adds to output row x = i (px = 0,
// u = j) or x = j (px = 1, u = i) the r-vector over y of sum_v S[y][v] M_t[u][v]
// (py = 2) or sum_v S[v][y] M_t[u][v] (py = 3).  One block per slab (i,j)
// stages the slab of each distinct T in LDS and writes two partial vectors,
// part[0][j][i][:] (px = 0 terms) and part[1][i][j][:] (px = 1 terms);
// k_contract42_reduce sums them over the slab's other index in a fixed order.
__global__ void __launch_bounds__(256)
k_contract42_slab(int r, SlabContractArgs a, double *__restrict__ part) {
  extern __shared__ double cs_smem[];
  const int rp = r + 1, r2 = r * r;
  const int q = blockIdx.x, i = q / r, j = q - (q / r) * r;
  const int y = threadIdx.x;
  double v0 = 0.0, v1 = 0.0;
  const double *staged = nullptr;
  for (int t = 0; t < a.nterms; ++t) {
    const SlabTerm &w = a.term[t];
    if (w.T != staged) {
      __syncthreads();  // every thread is done with the previous slab
      const double *src = w.T + (int64_t)q * r2;
      for (int e = threadIdx.x; e < r2; e += 256) cs_smem[(e / r) * rp + e % r] = src[e];
      __syncthreads();
      staged = w.T;
    }
    if (y < r) {
      const double *m = w.M + (w.px == 0 ? j : i) * r;
      double acc = 0.0;
      if (w.py == 2) {
        for (int v = 0; v < r; ++v) acc += cs_smem[y * rp + v] * m[v];
      } else {
        for (int v = 0; v < r; ++v) acc += cs_smem[v * rp + y] * m[v];
      }
      if (w.px == 0) v0 += w.c * acc; else v1 += w.c * acc;
    }
  }
  if (y < r) {
    part[((int64_t)j * r + i) * r + y] = v0;
    part[(int64_t)r2 * r + ((int64_t)i * r + j) * r + y] = v1;
  }
}

// out[x][y] (+)= sum_w part[0][w][x][y] + sum_w part[1][w][x][y]: 64 outputs
// per block, the 2r partials of each split over the 4 waves and summed in a
// fixed order.
__global__ void __launch_bounds__(256)
k_contract42_reduce(int r, const double *__restrict__ part, double *__restrict__ out, int accumulate) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r2 = r * r;
  const int e = blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (e < r2)
    for (int w = wave; w < 2 * r; w += 4) acc += part[(int64_t)w * r2 + e];  // part[0], then part[1]
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && e < r2) {
    const double v = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    out[e] = accumulate ? out[e] + v : v;
  }
}

// Particle-hole cotangents from S-bar:
//   E1b = -(S_aa - S_aa[j,i,k,l] - S_aa[i,j,l,k] + S_aa[j,i,l,k]),  sym = S_ab + S_ab[j,i,l,k]
//   P+b = E1b - sym,  P-b = E1b + sym,  E3b = sym
// One block per unordered pair {i <= j}, in two phases that each stage the
// rows (i,j) and (j,i) of one block in LDS (row stride r + 1) for the
// (k,l) <-> (l,k) reads: S_aa gives E1b (written to P+b and P-b), then S_ab
// gives sym (E3b, and P+-b updated in place).
__global__ void __launch_bounds__(512)
k_vjp_pe(int r, const double *__restrict__ Saa, const double *__restrict__ Sab,
         double *__restrict__ Ppb, double *__restrict__ Pmb, double *__restrict__ E3b) {
  extern __shared__ double pe_smem[];
  const int rp = r + 1, r2 = r * r;
  int i = 0, rem = blockIdx.x;
  while (rem >= r - i) { rem -= r - i; ++i; }
  const int j = i + rem;
  const int64_t ra = ((int64_t)i * r + j) * r2, rb = ((int64_t)j * r + i) * r2;
  double *Xa = pe_smem, *Xb = pe_smem + r * rp;
  auto stage = [&](const double *X) {
    for (int e = threadIdx.x; e < r2; e += 512) {
      const int k = e / r, l = e - (e / r) * r;
      Xa[k * rp + l] = X[ra + e];
      Xb[k * rp + l] = X[rb + e];
    }
  };
  stage(Saa);
  __syncthreads();
  for (int e = threadIdx.x; e < r2; e += 512) {
    const int k = e / r, l = e - (e / r) * r;
    const int n = k * rp + l, t = l * rp + k;
    const double e1a = -(Xa[n] - Xb[n] - Xa[t] + Xb[t]);
    Ppb[ra + e] = e1a;
    Pmb[ra + e] = e1a;
    if (i != j) {
      const double e1b = -(Xb[n] - Xa[n] - Xb[t] + Xa[t]);
      Ppb[rb + e] = e1b;
      Pmb[rb + e] = e1b;
    }
  }
  __syncthreads();
  stage(Sab);
  __syncthreads();
  for (int e = threadIdx.x; e < r2; e += 512) {
    const int k = e / r, l = e - (e / r) * r;
    const int n = k * rp + l, t = l * rp + k;
    const double sa = Xa[n] + Xb[t];
    Ppb[ra + e] -= sa;
    Pmb[ra + e] += sa;
    E3b[ra + e] = sa;
    if (i != j) {
      const double sb = Xb[n] + Xa[t];
      Ppb[rb + e] -= sb;
      Pmb[rb + e] += sb;
      E3b[rb + e] = sb;
    }
  }
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
// V-bar[p,r,q,s] = K_s-bar[p,q,r,s].  One block per (p,q): the A_aa-bar slab
// [p,q,:,:] is staged in LDS for its transposed read, and the block writes the
// r segments V-bar[p, rr, q, :].
__global__ void __launch_bounds__(256)
k_vjp_fold_v(int r, const double *__restrict__ Abaa, const double *__restrict__ Abab,
             double *__restrict__ Vb) {
  extern __shared__ double fv_smem[];
  const int rp = r + 1, r2 = r * r;
  const int p = blockIdx.x / r, q = blockIdx.x - (blockIdx.x / r) * r;
  const int64_t src = (int64_t)blockIdx.x * r2;  // [p,q,:,:]
  for (int e = threadIdx.x; e < r2; e += 256) {
    const int a = e / r, b = e - (e / r) * r;
    fv_smem[a * rp + b] = Abaa[src + e];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r2; e += 256) {
    const int rr = e / r, s = e - (e / r) * r;
    const double v = 0.5 * (fv_smem[rr * rp + s] - fv_smem[s * rp + rr]) + 0.5 * Abab[src + e];
    Vb[(((int64_t)p * r + rr) * r + q) * r + s] = v;
  }
}

// h-bar[p,r] = (sum_q K_s-bar[p,q,r,q] + sum_q K_s-bar[q,p,q,r]) / (N-1): one
// wavefront per output, lanes over q, fixed-order shuffle reduction.
__global__ void __launch_bounds__(256)
k_vjp_fold_h(int r, double inv_nm1, const double *__restrict__ Abaa, const double *__restrict__ Abab,
             double *__restrict__ hb) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= r * r) return;
  const int p = e / r, rr = e % r;
  const int64_t r2 = (int64_t)r * r;
  auto ks = [&](int a, int b, int c, int d) {
    const int64_t x = ((int64_t)a * r + b) * r2 + (int64_t)c * r + d;
    const int64_t y = ((int64_t)a * r + b) * r2 + (int64_t)d * r + c;
    return 0.5 * (Abaa[x] - Abaa[y]) + 0.5 * Abab[x];
  };
  double acc = 0.0;
  for (int q = lane; q < r; q += 64) acc += ks(p, q, rr, q) + ks(q, p, q, rr);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) hb[e] = acc * inv_nm1;
}

// Projections onto the symmetry subspaces of the inputs (scaled by c).
__global__ void k_proj_sym2(int r, double c, const double *__restrict__ x, double *__restrict__ out) {
  const int e = (int)vtid();
  if (e >= r * r) return;
  const int i = e / r, j = e % r;
  out[e] = c * 0.5 * (x[i * r + j] + x[j * r + i]);
}

// Projections of an r^4 gradient onto a symmetry subspace, in two passes.
// Pass 1 (k_proj_pairs), per unordered pair {i <= j}, combines the rows
// (i,j) and (j,i) of the r^2 x r^2 matrix and their (k,l) <-> (l,k) transposes:
//   y[ij,kl] = c0 x[ij,kl] + c1 x[ji,kl] + c2 x[ij,lk] + c3 x[ji,lk]
// (both rows staged in LDS, row stride r + 1).  Pass 2 (k_proj_exchange), in
// place: y <- c (y + y^T) / 2 under (ij) <-> (kl), on 32 x 32 tile pairs.
//   alpha-alpha 2-RDM block (antisymmetric pairs, Hermitian): c = (1, -1, -1, 1) / 4
//   V ((pq|rs), 8-fold):                                      c = (1, 1, 1, 1) / 4
//   alpha-beta 2-RDM block (Hermitian, (pq)(rs) -> (qp)(sr)):  c = (1, 0, 0, 1) / 2
__global__ void __launch_bounds__(256)
k_proj_pairs(int r, double c0, double c1, double c2, double c3, const double *__restrict__ x,
             double *__restrict__ y) {
  extern __shared__ double pp_smem[];
  const int rp = r + 1, r2 = r * r;
  int i = 0, rem = blockIdx.x;
  while (rem >= r - i) { rem -= r - i; ++i; }
  const int j = i + rem;
  const int64_t ra = ((int64_t)i * r + j) * r2, rb = ((int64_t)j * r + i) * r2;
  double *Xa = pp_smem, *Xb = pp_smem + r * rp;
  for (int e = threadIdx.x; e < r2; e += 256) {
    const int k = e / r, l = e - (e / r) * r;
    Xa[k * rp + l] = x[ra + e];
    Xb[k * rp + l] = x[rb + e];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r2; e += 256) {
    const int k = e / r, l = e - (e / r) * r;
    const double aa = Xa[k * rp + l], ba = Xb[k * rp + l], at = Xa[l * rp + k], bt = Xb[l * rp + k];
    y[ra + e] = c0 * aa + c1 * ba + c2 * at + c3 * bt;
    if (i != j) y[rb + e] = c0 * ba + c1 * aa + c2 * bt + c3 * at;
  }
}

constexpr int kPT = 32;  // exchange tile

__global__ void __launch_bounds__(256)
k_proj_exchange(int r, double c, double *__restrict__ y) {
  __shared__ double A[kPT][kPT + 1], B[kPT][kPT + 1];
  const int64_t r2 = (int64_t)r * r;
  const int nt = (int)((r2 + kPT - 1) / kPT);
  int tr, tc;
  unpair_le(nt, blockIdx.x, tr, tc);
  const int64_t R0 = (int64_t)tr * kPT, C0 = (int64_t)tc * kPT;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int q = 0; q < kPT; q += 8) {
    const int64_t ra = R0 + ty + q, ca = C0 + tx, rb = C0 + ty + q, cb = R0 + tx;
    A[ty + q][tx] = (ra < r2 && ca < r2) ? y[ra * r2 + ca] : 0.0;
    B[ty + q][tx] = (rb < r2 && cb < r2) ? y[rb * r2 + cb] : 0.0;
  }
  __syncthreads();
  const double h = 0.5 * c;
  for (int q = 0; q < kPT; q += 8) {
    const int64_t ra = R0 + ty + q, ca = C0 + tx, rb = C0 + ty + q, cb = R0 + tx;
    if (ra < r2 && ca < r2) y[ra * r2 + ca] = h * (A[ty + q][tx] + B[tx][ty + q]);
    if (tr != tc && rb < r2 && cb < r2) y[rb * r2 + cb] = h * (B[ty + q][tx] + A[tx][ty + q]);
  }
}

__global__ void k_identity(int r, double *__restrict__ I) {
  const int e = (int)vtid();
  if (e >= r * r) return;
  I[e] = (e / r == e % r) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// Form of a permute: q >= 0 the slice form moving position q (stage flags per
// source), q < 0 the row form.
static void permute_form(const PermArgs &a, int &q, int &stage1, int &stage2) {
  auto unit = [](const int64_t st[4]) {
    for (int p = 0; p < 3; ++p)
      if (st[p] == 1) return p;
    return -1;
  };
  q = -1;
  stage1 = stage2 = 0;
  const bool d1 = a.s1[3] == 1, d2 = !a.src2 || a.s2[3] == 1;
  if (!d1) {
    q = unit(a.s1);
    stage1 = 1;
    if (q >= 0 && !d2) {
      if (a.s2[q] == 1) stage2 = 1;
      else q = -1;
    }
  } else if (!d2) {
    q = unit(a.s2);
    stage2 = 1;
  }
}

static SliceStrides slice_strides(const PermArgs &a, int q, int stage1, int stage2) {
  // destination offset per unit of each index position (row = (0,1), col = (2,3))
  const int64_t os[4] = {(int64_t)a.r * a.ld, a.ld, a.r, 1};
  const int f1 = q == 0 ? 1 : 0, f2 = q == 2 ? 1 : 2;
  return SliceStrides{a.s1[f1], a.s1[f2], a.s1[q], a.s2[f1], a.s2[f2], a.s2[q],
                      os[q],    os[f1],   os[f2], stage1,   stage2};
}

template <class O>
static hipError_t launch_permute4_o(const PermArgs &a, int q, int stage1, int stage2, O out, hipStream_t s) {
  if (q < 0) {
    hipLaunchKernelGGL((k_permute4<O>), dim3((unsigned)a.rows), dim3(256), 0, s, a, out);
    return hipGetLastError();
  }
  const SliceStrides t = slice_strides(a, q, stage1, stage2);
  const size_t lds = (size_t)a.r * (a.r + 1) * sizeof(double);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_permute4_slice<O>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_permute4_slice<O>), dim3((unsigned)(a.r * a.r)), dim3(256), lds, s, a, t, out);
  const int64_t r2 = (int64_t)a.r * a.r;
  const int64_t npad = r2 * (a.ld - r2) + (a.rows - r2) * a.ld;
  if (!a.accumulate && npad > 0)
    hipLaunchKernelGGL((k_permute4_pad<O>), vgrid(npad), dim3(256), 0, s, a, out);
  return hipGetLastError();
}

hipError_t launch_permute4(GemmPrec prec, const PermArgs &a, const OperandRef &out, hipStream_t s) {
  // Slice form when a source's unit stride is not the destination's fast
  // position 3 but another position q < 3; a source whose unit stride is
  // position 3 is read directly.  Otherwise (all sources contiguous along
  // position 3, or two sources needing different slices) the row form.
  int q, stage1, stage2;
  permute_form(a, q, stage1, stage2);
  if (a.accumulate) {
    if (prec != GEMM_F64) return hipErrorInvalidValue;
    return launch_permute4_o(a, q, stage1, stage2, VOutF64Acc{static_cast<double *>(out.hi)}, s);
  }
  if (prec == GEMM_F64)
    return launch_permute4_o(a, q, stage1, stage2, VOutF64{static_cast<double *>(out.hi)}, s);
  if (prec == GEMM_F32)
    return launch_permute4_o(a, q, stage1, stage2, VOutF32{static_cast<float *>(out.hi)}, s);
  return launch_permute4_o(a, q, stage1, stage2,
                           VOutBF16x3{static_cast<__bf16 *>(out.hi), static_cast<__bf16 *>(out.lo)}, s);
}

// ---------------------------------------------------------------------------
// Pair packing and unpacking for the alpha-alpha pp adjoint products.  One
// thread per output element; a packed row's consecutive columns (c, d), c < d,
// run along d, so a source whose unit stride is position 3 is read in runs.
// ---------------------------------------------------------------------------
template <class O>
__global__ void __launch_bounds__(256)
k_pack_pairs(PairPackArgs a, int64_t rows, int64_t npk, O out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * a.ld) return;
  const int r = a.r;
  const int64_t m = e / a.ld;
  const int q = (int)(e - m * a.ld);
  double v = 0.0;
  if (q < npk) {
    int ia, ib, ic, id;
    if (a.rows_mode == 1) {
      unpair_lt(r, (int)m, ia, ib);
    } else if (a.rows_mode == 2) {
      unpair_le(r, (int)m, ia, ib);
    } else {
      ia = (int)(m / r);
      ib = (int)(m - (int64_t)ia * r);
    }
    if (a.k_le) unpair_le(r, q, ic, id);
    else unpair_lt(r, q, ic, id);
    for (int t = 0; t < a.nterms; ++t)
      if (!(a.offdiag[t] && ic == id))
        v += a.c[t] * a.src[t][ia * a.st[t][0] + ib * a.st[t][1] + ic * a.st[t][2] + id * a.st[t][3]];
  }
  out.put(e, v);
}

__global__ void __launch_bounds__(256)
k_unpack_pairs(int r, int rows_lt, const double *__restrict__ C, int64_t ldc, double *__restrict__ out) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= r2 * r2) return;
  const int64_t rowpq = e / r2, colrs = e - rowpq * r2;
  const int p = (int)(rowpq / r), q = (int)(rowpq - (int64_t)p * r);
  const int rr = (int)(colrs / r), ss = (int)(colrs - (int64_t)rr * r);
  double v = 0.0;
  if (rr != ss && !(rows_lt && p == q)) {
    const int64_t row = rows_lt ? pair_lt(r, min(p, q), max(p, q)) : rowpq;
    const int col = pair_lt(r, min(rr, ss), max(rr, ss));
    v = C[row * ldc + col];
    if (rr > ss) v = -v;
    if (rows_lt && p > q) v = -v;
  }
  out[e] = v;
}

hipError_t launch_pack_pairs(GemmPrec prec, const PairPackArgs &a, const OperandRef &out, hipStream_t s) {
  const int64_t npk = a.k_le ? npair_le(a.r) : npair_lt(a.r);
  if (a.nterms < 1 || a.nterms > 4 || a.ld < npk || a.rows_mode < 0 || a.rows_mode > 2) return hipErrorInvalidValue;
  const int64_t rows = a.rows_mode == 1 ? npair_lt(a.r) : a.rows_mode == 2 ? npair_le(a.r) : (int64_t)a.r * a.r;
  const dim3 grid = vgrid(rows * a.ld);
  if (prec == GEMM_F64)
    hipLaunchKernelGGL((k_pack_pairs<VOutF64>), grid, dim3(256), 0, s, a, rows, npk,
                       VOutF64{static_cast<double *>(out.hi)});
  else if (prec == GEMM_F32)
    hipLaunchKernelGGL((k_pack_pairs<VOutF32>), grid, dim3(256), 0, s, a, rows, npk,
                       VOutF32{static_cast<float *>(out.hi)});
  else
    hipLaunchKernelGGL((k_pack_pairs<VOutBF16x3>), grid, dim3(256), 0, s, a, rows, npk,
                       VOutBF16x3{static_cast<__bf16 *>(out.hi), static_cast<__bf16 *>(out.lo)});
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
k_unpack_pm(int r, int rows_packed, const double *__restrict__ Cp, int64_t ldp, const double *__restrict__ Cm,
            int64_t ldm, double *__restrict__ out) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= r2 * r2) return;
  const int64_t rowpq = e / r2, colrs = e - rowpq * r2;
  const int p = (int)(rowpq / r), q = (int)(rowpq - (int64_t)p * r);
  const int rr = (int)(colrs / r), ss = (int)(colrs - (int64_t)rr * r);
  const int a = min(p, q), b = max(p, q), c = min(rr, ss), d = max(rr, ss);
  const int64_t rowp = rows_packed ? pair_le(r, a, b) : rowpq;
  double v = Cp[rowp * ldp + pair_le(r, c, d)];
  if (c != d && !(rows_packed && a == b)) {
    const int64_t rowm = rows_packed ? pair_lt(r, a, b) : rowpq;
    double w = Cm[rowm * ldm + pair_lt(r, c, d)];
    if (rr > ss) w = -w;
    if (rows_packed && p > q) w = -w;
    v += w;
  }
  out[e] = 0.5 * v;
}

hipError_t launch_unpack_pm(int r, int rows_packed, const double *Cp, int64_t ldp, const double *Cm, int64_t ldm,
                            double *out, hipStream_t s) {
  const int64_t r2 = (int64_t)r * r;
  hipLaunchKernelGGL(k_unpack_pm, vgrid(r2 * r2), dim3(256), 0, s, r, rows_packed, Cp, ldp, Cm, ldm, out);
  return hipGetLastError();
}

hipError_t launch_unpack_pairs(int r, int rows_lt, const double *C, int64_t ldc, double *out, hipStream_t s) {
  const int64_t r2 = (int64_t)r * r;
  hipLaunchKernelGGL(k_unpack_pairs, vgrid(r2 * r2), dim3(256), 0, s, r, rows_lt, C, ldc, out);
  return hipGetLastError();
}

hipError_t launch_contract42(int r, const ContractArgs &a, double *out, int accumulate, double *part,
                             hipStream_t s) {
  // slab form when every term has x, u in the first index pair and y, v in the
  // second (strides of the natural r^4 layout)
  const int64_t S[4] = {(int64_t)r * r * r, (int64_t)r * r, r, 1};
  SlabContractArgs b{};
  bool slab = part != nullptr && r <= 256;
  for (int t = 0; t < a.nterms && slab; ++t) {
    const ContractTerm &q = a.term[t];
    const bool x0 = q.sx == S[0] && q.su == S[1], x1 = q.sx == S[1] && q.su == S[0];
    const bool y2 = q.sy == S[2] && q.sv == S[3], y3 = q.sy == S[3] && q.sv == S[2];
    if (!(x0 || x1) || !(y2 || y3)) { slab = false; break; }
    b.term[t] = SlabTerm{q.T, q.M, q.c, x0 ? 0 : 1, y2 ? 2 : 3};
  }
  if (!slab) {
    hipLaunchKernelGGL(k_contract42, dim3((unsigned)(r * r)), dim3(256), 0, s, r, a, out, accumulate);
    return hipGetLastError();
  }
  b.nterms = a.nterms;
  const size_t lds = (size_t)r * (r + 1) * sizeof(double);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_contract42_slab),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_contract42_slab, dim3((unsigned)(r * r)), dim3(256), lds, s, r, b, part);
  hipLaunchKernelGGL(k_contract42_reduce, dim3((unsigned)((r * r + 63) / 64)), dim3(256), 0, s, r, part, out,
                     accumulate);
  return hipGetLastError();
}

hipError_t launch_vjp_pe(int r, const double *Saa, const double *Sab, double *Ppb, double *Pmb,
                         double *E3b, hipStream_t s) {
  const size_t lds = (size_t)2 * r * (r + 1) * sizeof(double);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_vjp_pe),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vjp_pe, dim3((unsigned)(r * (r + 1) / 2)), dim3(512), lds, s, r, Saa, Sab, Ppb, Pmb,
                     E3b);
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
  const size_t lds = (size_t)r * (r + 1) * sizeof(double);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_vjp_fold_v),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_vjp_fold_v, dim3((unsigned)(r * r)), dim3(256), lds, s, r, Abaa, Abab, Vb_raw);
  hipLaunchKernelGGL(k_vjp_fold_h, dim3((unsigned)((r * r + 3) / 4)), dim3(256), 0, s, r, 1.0 / (N - 1), Abaa,
                     Abab, hb_raw);
  return hipGetLastError();
}

hipError_t launch_proj(ProjKind k, int r, double c, const double *x, double *out, hipStream_t s) {
  if (k == PROJ_SYM2) {
    hipLaunchKernelGGL(k_proj_sym2, vgrid((int64_t)r * r), dim3(256), 0, s, r, c, x, out);
    return hipGetLastError();
  }
  double c4[4];
  if (k == PROJ_AA) { c4[0] = 0.25; c4[1] = -0.25; c4[2] = -0.25; c4[3] = 0.25; }
  else if (k == PROJ_V) { c4[0] = c4[1] = c4[2] = c4[3] = 0.25; }
  else { c4[0] = 0.5; c4[1] = 0.0; c4[2] = 0.0; c4[3] = 0.5; }
  const size_t lds = (size_t)2 * r * (r + 1) * sizeof(double);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_proj_pairs),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_proj_pairs, dim3((unsigned)(r * (r + 1) / 2)), dim3(256), lds, s, r, c4[0], c4[1], c4[2],
                     c4[3], x, out);
  const int nt = (r * r + kPT - 1) / kPT;
  hipLaunchKernelGGL(k_proj_exchange, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s, r, c, out);
  return hipGetLastError();
}

hipError_t launch_identity(int r, double *I, hipStream_t s) {
  hipLaunchKernelGGL(k_identity, vgrid((int64_t)r * r), dim3(256), 0, s, r, I);
  return hipGetLastError();
}

}  // namespace acse

namespace acse {

template <class O>
static hipError_t launch_batch_o(const PermArgs *a, const O *out, int count, hipStream_t s) {
  PermBatch<O> b{};
  b.count = count;
  int nmain = 0, npadb = 0, r = 0;
  bool any_slice = false;
  for (int j = 0; j < count; ++j) {
    int q, st1, st2;
    permute_form(a[j], q, st1, st2);
    b.a[j] = a[j];
    b.out[j] = out[j];
    b.slice[j] = q >= 0;
    if (q >= 0) b.t[j] = slice_strides(a[j], q, st1, st2);
    b.start[j] = nmain;
    nmain += q >= 0 ? a[j].r * a[j].r : (int)a[j].rows;
    r = std::max(r, a[j].r);
    any_slice = any_slice || q >= 0;
  }
  b.start[count] = nmain;
  for (int j = 0; j < count; ++j) {
    b.pstart[j] = npadb;
    if (b.slice[j] && !a[j].accumulate) {
      const int64_t r2 = (int64_t)a[j].r * a[j].r;
      const int64_t npad = r2 * (a[j].ld - r2) + (a[j].rows - r2) * a[j].ld;
      npadb += (int)((npad + 255) / 256);
    }
  }
  b.pstart[count] = npadb;
  const size_t lds = any_slice ? (size_t)r * (r + 1) * sizeof(double) : 0;
  if (lds) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_permute4_batch<O>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_permute4_batch<O>), dim3((unsigned)(nmain + npadb)), dim3(256), lds, s, b);
  return hipGetLastError();
}

hipError_t launch_permute4_batch(const GemmPrec *prec, const PermArgs *a, const OperandRef *out, int count,
                                 hipStream_t s) {
  // consecutive jobs of one destination type go out together
  for (int j0 = 0; j0 < count;) {
    const bool acc = a[j0].accumulate != 0;
    const GemmPrec p = prec[j0];
    if (acc && p != GEMM_F64) return hipErrorInvalidValue;
    int j1 = j0 + 1;
    while (j1 < count && j1 - j0 < kMaxPermJobs && prec[j1] == p && (a[j1].accumulate != 0) == acc) ++j1;
    const int n = j1 - j0;
    hipError_t e = hipSuccess;
    if (acc) {
      VOutF64Acc o[kMaxPermJobs];
      for (int j = 0; j < n; ++j) o[j] = VOutF64Acc{static_cast<double *>(out[j0 + j].hi)};
      e = launch_batch_o(a + j0, o, n, s);
    } else if (p == GEMM_F64) {
      VOutF64 o[kMaxPermJobs];
      for (int j = 0; j < n; ++j) o[j] = VOutF64{static_cast<double *>(out[j0 + j].hi)};
      e = launch_batch_o(a + j0, o, n, s);
    } else if (p == GEMM_F32) {
      VOutF32 o[kMaxPermJobs];
      for (int j = 0; j < n; ++j) o[j] = VOutF32{static_cast<float *>(out[j0 + j].hi)};
      e = launch_batch_o(a + j0, o, n, s);
    } else {
      VOutBF16x3 o[kMaxPermJobs];
      for (int j = 0; j < n; ++j)
        o[j] = VOutBF16x3{static_cast<__bf16 *>(out[j0 + j].hi), static_cast<__bf16 *>(out[j0 + j].lo)};
      e = launch_batch_o(a + j0, o, n, s);
    }
    if (e != hipSuccess) return e;
    j0 = j1;
  }
  return hipSuccess;
}

}  // namespace acse
