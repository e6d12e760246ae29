// Generic O(r^4) kernels of the general-spin residual map: linear
// combinations of index-permuted spin blocks, GEMM operand packing, outer
// products of two-index tensors, partial traces and the per-block step tail.
// The O(r^6) work of the map runs on the grouped MFMA GEMM and the O(r^5)
// one-index transforms on the mode-product kernel (tensor_ops.hip).
#include "spin.h"

namespace acse {

namespace {

__device__ inline bool all_active(const ActiveBits &m, int i, int j, int k, int l) {
  auto on = [&](int q) { return (m.w[q >> 6] >> (q & 63)) & 1ull; };
  return on(i) && on(j) && on(k) && on(l);
}

// One thread per output element; the output is written in its natural order
// (coalesced), the terms are read through their strides.
__global__ void __launch_bounds__(256)
k_combine4(int r, const Terms4 T, double *__restrict__ out, int accumulate, int masked, const ActiveBits mask) {
  const int64_t n = (int64_t)r * r * r * r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int l = (int)(e % r), k = (int)((e / r) % r), j = (int)((e / ((int64_t)r * r)) % r),
            i = (int)(e / ((int64_t)r * r * r));
  double v = 0.0;
  for (int t = 0; t < T.n; ++t) {
    const Term4 &q = T.t[t];
    v += q.c * q.in[i * q.s[0] + j * q.s[1] + k * q.s[2] + l * q.s[3]];
  }
  if (accumulate) v += out[e];
  if (masked && all_active(mask, i, j, k, l)) v = 0.0;
  out[e] = v;
}

__global__ void __launch_bounds__(256) k_pack_op4(int r, const Terms4 T, double *__restrict__ out, int ld) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= r2 * ld) return;
  const int64_t row = e / ld, col = e - row * ld;
  double v = 0.0;
  if (col < r2) {
    const int i = (int)(row / r), j = (int)(row % r), k = (int)(col / r), l = (int)(col % r);
    for (int t = 0; t < T.n; ++t) {
      const Term4 &q = T.t[t];
      v += q.c * q.in[i * q.s[0] + j * q.s[1] + k * q.s[2] + l * q.s[3]];
    }
  }
  out[e] = v;
}

__global__ void __launch_bounds__(256)
k_outer4(int r, double c, const double *__restrict__ A, int a0, int a1, const double *__restrict__ B, int b0, int b1,
         double *__restrict__ out) {
  const int64_t n = (int64_t)r * r * r * r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  int x[4];
  x[3] = (int)(e % r);
  x[2] = (int)((e / r) % r);
  x[1] = (int)((e / ((int64_t)r * r)) % r);
  x[0] = (int)(e / ((int64_t)r * r * r));
  out[e] += c * A[x[a0] * r + x[a1]] * B[x[b0] * r + x[b1]];
}

__global__ void k_trace12(int r, const double *__restrict__ in, double *__restrict__ out, int accumulate) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * r) return;
  const int k = e / r, s = e % r;
  const int64_t r2 = (int64_t)r * r, r3 = r2 * r;
  double v = 0.0;
  for (int q = 0; q < r; ++q) v += in[k * r3 + q * r2 + q * r + s];
  out[e] = accumulate ? out[e] + v : v;
}

struct TraceArgs {
  const double *in[8];
};

// One block per array: sum over the r^2 diagonal pairs in a fixed order.
__global__ void __launch_bounds__(256) k_pair_traces(int r, const TraceArgs a, double *traces) {
  __shared__ double red[256];
  const double *in = a.in[blockIdx.x];
  const int64_t r2 = (int64_t)r * r;
  double v = 0.0;
  for (int64_t pq = threadIdx.x; pq < r2; pq += 256) v += in[pq * r2 + pq];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) traces[blockIdx.x] = red[0];
}

struct UpdateArgs {
  double *d2[3];
  const double *U[3];
};

__global__ void __launch_bounds__(256) k_spin_update(int r, double eps, const UpdateArgs a, const double *traces) {
  const int64_t n = (int64_t)r * r * r * r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int q = blockIdx.y;
  if (e >= n) return;
  const double t0 = traces[q], tu = traces[3 + q];
  // a block with zero input trace (fewer than two electrons of its pair kind)
  // is set to zero
  const double scale = t0 != 0.0 ? t0 / (t0 + eps * tu) : 0.0;
  a.d2[q][e] = (a.d2[q][e] + eps * a.U[q][e]) * scale;
}

__global__ void k_spin_1rdm(int r, double c, const double *__restrict__ aa, const double *__restrict__ bb,
                            const double *__restrict__ ab, double *__restrict__ ga, double *__restrict__ gb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= r * r) return;
  const int p = e / r, s = e % r;
  const int64_t r2 = (int64_t)r * r, r3 = r2 * r;
  double va = 0.0, vb = 0.0;
  for (int q = 0; q < r; ++q) {
    va += aa[p * r3 + q * r2 + s * r + q] + ab[p * r3 + q * r2 + s * r + q];   // 2D(pa q|sa q)
    vb += bb[p * r3 + q * r2 + s * r + q] + ab[q * r3 + p * r2 + q * r + s];   // 2D(pb q|sb q)
  }
  ga[e] = c * va;
  gb[e] = c * vb;
}

// out[i,j,k,l] = sign(i,j) C[pair(min(i,j), max(i,j))][k r + l], zero for i = j.
__global__ void __launch_bounds__(256)
k_unpack_rows_lt(int r, const double *__restrict__ C, int64_t ldc, double *__restrict__ out) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= r2 * r2) return;
  const int64_t row = e / r2, col = e - row * r2;
  const int i = (int)(row / r), j = (int)(row - (int64_t)i * r);
  double v = 0.0;
  if (i != j) {
    v = C[(int64_t)pair_lt(r, min(i, j), max(i, j)) * ldc + col];
    if (i > j) v = -v;
  }
  out[e] = v;
}

// One thread per spatial element of the block; the writes of a thread run
// along l (contiguous in the block of the output).
__global__ void __launch_bounds__(256)
k_so_embed(int r, int bits, const double *__restrict__ in, double c, double *__restrict__ out) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= r2 * r2) return;
  const int l = (int)(e % r), k = (int)((e / r) % r), j = (int)((e / r2) % r), i = (int)(e / (r2 * r));
  const int64_t n = 2 * (int64_t)r;
  const int i2 = i + (((bits >> 3) & 1) ? r : 0), j2 = j + (((bits >> 2) & 1) ? r : 0);
  const int k2 = k + (((bits >> 1) & 1) ? r : 0), l2 = l + ((bits & 1) ? r : 0);
  out[((i2 * n + j2) * n + k2) * n + l2] = c * in[e];
}

// One thread per spin-orbital element (I,J,A,B).
__global__ void __launch_bounds__(256)
k_so_cumulant(int r, const double *__restrict__ ga, const double *__restrict__ gb, const double *__restrict__ d2aa,
              const double *__restrict__ d2bb, const double *__restrict__ d2ab, const double *__restrict__ sig,
              double *__restrict__ c2, double *__restrict__ cs) {
  const int64_t n = 2 * (int64_t)r, n2 = n * n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n2 * n2) return;
  const int B = (int)(e % n), A = (int)((e / n) % n), J = (int)((e / n2) % n), I = (int)(e / (n2 * n));
  const int si = I >= r, sj = J >= r, sa = A >= r, sb = B >= r;
  const int i = I - si * r, j = J - sj * r, a = A - sa * r, b = B - sb * r;
  const int64_t r2 = (int64_t)r * r;
  auto at = [&](int p, int q, int u, int v) { return ((int64_t)p * r + q) * r2 + (int64_t)u * r + v; };
  // 2D from the blocks: the fixed-spin blocks and the three mixed ones by the
  // antisymmetry of each index pair; zero unless the spins of (I,J) are those of (A,B)
  double d = 0.0;
  const int code = (si << 3) | (sj << 2) | (sa << 1) | sb;
  switch (code) {
    case 0x0: d = d2aa[at(i, j, a, b)]; break;
    case 0xF: d = d2bb[at(i, j, a, b)]; break;
    case 0x5: d = d2ab[at(i, j, a, b)]; break;
    case 0xA: d = d2ab[at(j, i, b, a)]; break;
    case 0x6: d = -d2ab[at(i, j, b, a)]; break;
    case 0x9: d = -d2ab[at(j, i, a, b)]; break;
    default: break;
  }
  // 1D spin-diagonal
  auto g1 = [&](int p, int sp, int q, int sq) -> double {
    if (sp != sq) return 0.0;
    return (sp ? gb : ga)[(int64_t)p * r + q];
  };
  const double v = d - 0.5 * (g1(i, si, a, sa) * g1(j, sj, b, sb) - g1(j, sj, a, sa) * g1(i, si, b, sb));
  c2[e] = v;
  cs[e] = sig[A] * v;
}

// One thread per (k,a): the sum over p in a fixed order.
__global__ void __launch_bounds__(256) k_so_trace_y(int n, const double *__restrict__ W, double *__restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int k = (int)(e / n), a = (int)(e % n);
  const int64_t n2 = (int64_t)n * n;
  double acc = 0.0;
  for (int p = 0; p < n; ++p) acc += W[((int64_t)k * n + p) * n2 + (int64_t)p * n + a];
  Y[e] = acc;
}

// t_pl: B[i,j,k,l] += c sum_a Y[k,a] cs[i,j,a,l].  Y and cs conserve spin
// (Y_ka is zero unless a has the spin of k), so for given (i, j, l) only k and
// a of the one spin sk = s_i + s_j - s_l contribute (none unless sk is 0 or
// 1).  One thread per (i, j, l) keeps the r results of its k block in
// registers; the two same-spin blocks of Y, transposed ([a][k]), sit in LDS
// (2 r^2 doubles, 64 KB at r = 64); each conserving cs element is read once
// and each output read and written once; the sum over a runs in a fixed
// order.
constexpr int kTplMaxR = 64;
__global__ void __launch_bounds__(256)
k_so_tpl(int n, double c, const double *__restrict__ Y, const double *__restrict__ cs, double *__restrict__ B) {
  extern __shared__ double tpl_yt[];  // [spin][a][k] = Y[spin r + k][spin r + a]
  const int r = n / 2;
  const int rr = r * r;
  for (int e = threadIdx.x; e < 2 * rr; e += 256) {
    const int sp = e / rr, q = e - sp * rr, a = q / r, k = q - a * r;
    tpl_yt[e] = Y[(int64_t)(sp * r + k) * n + sp * r + a];
  }
  __syncthreads();
  const int64_t n2 = (int64_t)n * n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n2 * n) return;
  const int l = (int)(e % n);
  const int64_t ij = e / n;
  const int i = (int)(ij / n), j = (int)(ij % n);
  const int sk = (i >= r) + (j >= r) - (l >= r);
  if (sk < 0 || sk > 1) return;
  const double *q = cs + ij * n2 + (int64_t)sk * r * n + l;
  const double *yb = tpl_yt + sk * rr;
  double acc[kTplMaxR];
#pragma unroll
  for (int t = 0; t < kTplMaxR; ++t) acc[t] = 0.0;
  for (int a = 0; a < r; ++a) {
    const double v = q[(int64_t)a * n];
    const double *ya = yb + a * r;
#pragma unroll
    for (int t = 0; t < kTplMaxR; ++t)
      if (t < r) acc[t] += ya[t] * v;
  }
  double *bo = B + ij * n2 + (int64_t)sk * r * n + l;
#pragma unroll
  for (int t = 0; t < kTplMaxR; ++t)
    if (t < r) bo[(int64_t)t * n] += c * acc[t];
}

// One workgroup per (letter values of the two positions other than u and 3),
// looping over the 32 x 32 tiles of positions u and 3, u the operand position
// the source reads with unit stride: a tile is read along u and written along
// position 3 through LDS.  If the source's unit stride is position 3 itself
// (u = 3), tiles are read and written along position 3 directly.  Addresses
// are sums of per-position terms: letter value L of operand position t adds
// L b[t] + (L >= r) (o[t] - r b[t]) to the destination offset and L st[t] to
// the source offset; the source element conserves spin iff
// sum_t c[t] (L_t >= r) = 0.
struct SoPackArgs {
  int64_t st[4];   // source strides of the operand positions
  int64_t b[4];    // destination offset per unit of the spatial index of each position
  int64_t o[4];    // destination offset of a beta letter at each position
  int c[4];        // +1 / -1: the side of the source's conservation pair each position is on
  int u, v, w;     // u: the unit-stride position (3: none other); v, w: the fixed ones
};
__global__ void __launch_bounds__(256)
k_so_pack(int r, const double *__restrict__ src, SoPackArgs a, double *__restrict__ out) {
  __shared__ double tile[32][33];
  const int n = 2 * r;
  const int nt = (n + 31) / 32;
  const int Lw = blockIdx.x % n, Lv = blockIdx.x / n;
  auto off = [&](int t, int L) { return L * a.b[t] + (L >= r ? a.o[t] - r * a.b[t] : 0); };
  const int64_t obase = off(a.v, Lv) + off(a.w, Lw);
  const int64_t sbase = Lv * a.st[a.v] + Lw * a.st[a.w];
  const int cbase = a.c[a.v] * (Lv >= r) + a.c[a.w] * (Lw >= r);
  if (a.u == 3) {
    // the third free position (the one of 0..2 other than v, w) and position 3
    const int third = 3 - a.v - a.w;
    for (int tt = 0; tt < nt * nt; ++tt) {
      const int tu = tt / nt, t3 = tt % nt;
      for (int q = threadIdx.x; q < 32 * 32; q += 256) {
        const int Lt = tu * 32 + q / 32, L3 = t3 * 32 + q % 32;
        if (Lt >= n || L3 >= n) continue;
        if (cbase + a.c[third] * (Lt >= r) + a.c[3] * (L3 >= r) != 0) continue;
        out[obase + off(third, Lt) + off(3, L3)] = src[sbase + Lt * a.st[third] + L3];
      }
    }
    return;
  }
  for (int tt = 0; tt < nt * nt; ++tt) {
    const int tu = tt / nt, t3 = tt % nt;
    __syncthreads();  // the previous tile's reads of LDS are done
    for (int q = threadIdx.x; q < 32 * 32; q += 256) {
      const int Lu = tu * 32 + q % 32, L3 = t3 * 32 + q / 32;
      const bool ok = Lu < n && L3 < n && cbase + a.c[a.u] * (Lu >= r) + a.c[3] * (L3 >= r) == 0;
      tile[q / 32][q % 32] = ok ? src[sbase + Lu + L3 * a.st[3]] : 0.0;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 32 * 32; q += 256) {
      const int Lu = tu * 32 + q / 32, L3 = t3 * 32 + q % 32;
      if (Lu >= n || L3 >= n) continue;
      if (cbase + a.c[a.u] * (Lu >= r) + a.c[3] * (L3 >= r) != 0) continue;
      out[obase + off(a.u, Lu) + off(3, L3)] = tile[q % 32][q / 32];
    }
  }
}

// ---- adjoint of the NY share on singlet states ------------------------------
__global__ void __launch_bounds__(256)
k_so_embed_singlet_x(int r, const double *__restrict__ Aaa, const double *__restrict__ Aab, double *__restrict__ X) {
  const int64_t n = 2 * (int64_t)r, n2 = n * n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n2 * n2) return;
  const int L = (int)(e % n), K = (int)((e / n) % n), J = (int)((e / n2) % n), I = (int)(e / (n2 * n));
  const int si = I >= r, sj = J >= r, sk = K >= r, sl = L >= r;
  const int i = I - si * r, j = J - sj * r, k = K - sk * r, l = L - sl * r;
  const int64_t r2 = (int64_t)r * r;
  const int64_t nat = ((int64_t)i * r + j) * r2 + (int64_t)k * r + l;
  const int64_t swp = ((int64_t)i * r + j) * r2 + (int64_t)l * r + k;
  double v = 0.0;
  switch ((si << 3) | (sj << 2) | (sk << 1) | sl) {
    case 0x0: case 0xF: v = Aaa[nat]; break;
    case 0x5: case 0xA: v = Aab[nat]; break;
    case 0x6: case 0x9: v = -Aab[swp]; break;
    default: break;
  }
  X[e] = v;
}

__global__ void __launch_bounds__(256)
k_so_xbar_singlet(int r, const double *__restrict__ Xb, double *__restrict__ Abaa, double *__restrict__ Abab) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= r2 * r2) return;
  const int l = (int)(e % r), k = (int)((e / r) % r), j = (int)((e / r2) % r), i = (int)(e / (r2 * r));
  const int64_t n = 2 * (int64_t)r;
  auto at = [&](int a, int b, int c, int d) { return Xb[((a * n + b) * n + c) * n + d]; };
  Abaa[e] += at(i, j, k, l) + at(i + r, j + r, k + r, l + r);
  Abab[e] += at(i, j + r, k, l + r) + at(i + r, j, k + r, l) - at(i, j + r, l + r, k) - at(i + r, j, l, k + r);
}

__global__ void __launch_bounds__(256)
k_so_dbar_singlet(int r, double c, const double *__restrict__ D, double *__restrict__ Gaa, double *__restrict__ Gab) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= r2 * r2) return;
  // output element [p,q,u,t]
  const int t = (int)(e % r), u = (int)((e / r) % r), q = (int)((e / r2) % r), p = (int)(e / (r2 * r));
  const int64_t n = 2 * (int64_t)r;
  auto at = [&](int w, int x, int y, int z) { return D[((w * n + x) * n + y) * n + z]; };
  Gaa[e] += c * (at(p, q, u, t) + at(p + r, q + r, u + r, t + r));
  Gab[e] += c * (at(p, q + r, u, t + r) + at(q + r, p, t + r, u) - at(p, q + r, t + r, u) -
                 at(q + r, p, u, t + r));
}

__global__ void __launch_bounds__(256)
k_so_bbar(int r, const double *__restrict__ Raa, const double *__restrict__ Rab, double sign, double *__restrict__ Bb) {
  const int64_t n = 2 * (int64_t)r, n2 = n * n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n2 * n2) return;
  const int L = (int)(e % n), K = (int)((e / n) % n), J = (int)((e / n2) % n), I = (int)(e / (n2 * n));
  const int64_t r2 = (int64_t)r * r;
  // the cotangent of the spin-orbital residual: Rbar_aa on (aa|aa), Rbar_ab on (ab|ab)
  auto rb = [&](int a, int b, int c, int d) -> double {
    const int sa = a >= r, sb = b >= r, sc = c >= r, sd = d >= r;
    const int64_t x = ((int64_t)(a - sa * r) * r + (b - sb * r)) * r2 + (int64_t)(c - sc * r) * r + (d - sd * r);
    const int code = (sa << 3) | (sb << 2) | (sc << 1) | sd;
    return code == 0 ? Raa[x] : code == 5 ? Rab[x] : 0.0;
  };
  Bb[e] = -rb(I, J, K, L) + rb(I, J, L, K) + sign * (rb(K, L, I, J) - rb(L, K, I, J));
}

// Ybar[k,a] = c sum_{i,j,l} Bbar[i,j,k,l] cs[i,j,a,l] over the conserving
// elements: a and k share one spin sa, and for given (i, j) the spin of l is
// s_i + s_j - sa.  Split over (i, j): workgroup w takes a contiguous range of
// (i, j) and, per spin case, stages the r x r blocks Bbar[i,j,sa.,sl.] and
// cs[i,j,sa.,sl.] in LDS (rows padded to r + 1), each thread accumulating up
// to two 4 x 4 register blocks of its partial Ybar (both spin blocks, 2 r^2
// values per workgroup); a second pass sums the partials over the workgroups
// in a fixed order.  Every conserving Bbar and cs element is read once.
constexpr int kYbB = 4;
__global__ void __launch_bounds__(256)
k_so_ybar_part(int n, const double *__restrict__ Bb, const double *__restrict__ cs, double *__restrict__ part) {
  extern __shared__ double ybar_s[];
  const int r = n / 2, rp = r + 1, nb = (r + kYbB - 1) / kYbB, nblk = 2 * nb * nb;
  double *const TB = ybar_s, *const CB = ybar_s + r * rp;
  const int64_t n2 = (int64_t)n * n;
  const int64_t ij0 = n2 * blockIdx.x / gridDim.x, ij1 = n2 * (blockIdx.x + 1) / gridDim.x;
  double acc[2][kYbB][kYbB];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int u = 0; u < kYbB; ++u)
#pragma unroll
      for (int v = 0; v < kYbB; ++v) acc[q][u][v] = 0.0;
  for (int64_t ij = ij0; ij < ij1; ++ij) {
    const int i = (int)(ij / n), j = (int)(ij % n);
    const int st = (i >= r) + (j >= r);
    for (int sa = 0; sa < 2; ++sa) {
      const int sl = st - sa;
      if (sl < 0 || sl > 1) continue;  // the same for the whole workgroup
      __syncthreads();                 // the previous blocks are fully read
      const double *tb = Bb + ij * n2 + (int64_t)sa * r * n + sl * r;
      const double *cb = cs + ij * n2 + (int64_t)sa * r * n + sl * r;
      for (int e = threadIdx.x; e < r * r; e += 256) {
        const int x = e / r, l = e - x * r;
        TB[x * rp + l] = tb[(int64_t)x * n + l];
        CB[x * rp + l] = cb[(int64_t)x * n + l];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int bb = threadIdx.x + 256 * q;
        if (bb >= nblk || bb / (nb * nb) != sa) continue;
        const int k0 = ((bb % (nb * nb)) / nb) * kYbB, a0 = (bb % nb) * kYbB;
        for (int l = 0; l < r; ++l) {
          double tv[kYbB], cv[kYbB];
#pragma unroll
          for (int u = 0; u < kYbB; ++u) {
            tv[u] = k0 + u < r ? TB[(k0 + u) * rp + l] : 0.0;
            cv[u] = a0 + u < r ? CB[(a0 + u) * rp + l] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kYbB; ++u)
#pragma unroll
            for (int v = 0; v < kYbB; ++v) acc[q][u][v] += tv[u] * cv[v];
        }
      }
    }
  }
  double *po = part + (int64_t)blockIdx.x * 2 * r * r;  // [spin][k][a]
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int bb = threadIdx.x + 256 * q;
    if (bb >= nblk) continue;
    const int sa = bb / (nb * nb), k0 = ((bb % (nb * nb)) / nb) * kYbB, a0 = (bb % nb) * kYbB;
#pragma unroll
    for (int u = 0; u < kYbB; ++u)
#pragma unroll
      for (int v = 0; v < kYbB; ++v)
        if (k0 + u < r && a0 + v < r) po[((int64_t)sa * r + k0 + u) * r + a0 + v] = acc[q][u][v];
  }
}

// Ybar = c x the sum of the partials in workgroup order; zero between spins.
__global__ void __launch_bounds__(256)
k_so_ybar_sum(int n, double c, const double *__restrict__ part, int nparts, double *__restrict__ Yb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int r = n / 2;
  const int k = (int)(e / n), a = (int)(e % n);
  const int sk = k >= r;
  if ((a >= r) != sk) {
    Yb[e] = 0.0;
    return;
  }
  const int64_t o = ((int64_t)sk * r + (k - sk * r)) * r + (a - sk * r), stride = 2 * (int64_t)r * r;
  double acc = 0.0;
  for (int w = 0; w < nparts; ++w) acc += part[w * stride + o];
  Yb[e] = c * acc;
}

// csbar[i,j,a,l] += c sum_k Bbar[i,j,k,l] Y[k,a] over the conserving
// elements: for given (i, j, l) the spin sa = s_i + s_j - s_l of a (none
// unless 0 or 1) is also k's (Y conserves spin).  One thread per (i, j, l)
// keeps the r results of its a block in registers, Y's two same-spin blocks
// ([k][a]) sit in LDS, and each conserving Bbar element is read once; the sum
// over k runs in a fixed order.
__global__ void __launch_bounds__(256)
k_so_csbar_pl(int n, double c, const double *__restrict__ Bb, const double *__restrict__ Y, double *__restrict__ CSb) {
  extern __shared__ double csb_y[];  // [spin][k][a] = Y[spin r + k][spin r + a]
  const int r = n / 2;
  const int rr = r * r;
  for (int e = threadIdx.x; e < 2 * rr; e += 256) {
    const int sp = e / rr, q = e - sp * rr, k = q / r, a = q - k * r;
    csb_y[e] = Y[(int64_t)(sp * r + k) * n + sp * r + a];
  }
  __syncthreads();
  const int64_t n2 = (int64_t)n * n;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n2 * n) return;
  const int l = (int)(e % n);
  const int64_t ij = e / n;
  const int i = (int)(ij / n), j = (int)(ij % n);
  const int sa = (i >= r) + (j >= r) - (l >= r);
  if (sa < 0 || sa > 1) return;
  const double *b = Bb + ij * n2 + (int64_t)sa * r * n + l;
  const double *yb = csb_y + sa * rr;
  double acc[kTplMaxR];
#pragma unroll
  for (int t = 0; t < kTplMaxR; ++t) acc[t] = 0.0;
  for (int k = 0; k < r; ++k) {
    const double v = b[(int64_t)k * n];
    const double *yk = yb + k * r;
#pragma unroll
    for (int t = 0; t < kTplMaxR; ++t)
      if (t < r) acc[t] += v * yk[t];
  }
  double *o = CSb + ij * n2 + (int64_t)sa * r * n + l;
#pragma unroll
  for (int t = 0; t < kTplMaxR; ++t)
    if (t < r) o[(int64_t)t * n] += c * acc[t];
}

__global__ void __launch_bounds__(256) k_so_diag_add(int n, const double *__restrict__ Yb, double *__restrict__ Wb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n * n) return;
  const int a = (int)(e % n), p = (int)((e / n) % n), k = (int)(e / ((int64_t)n * n));
  const int64_t n2 = (int64_t)n * n;
  Wb[((int64_t)k * n + p) * n2 + (int64_t)p * n + a] += Yb[(int64_t)k * n + a];
}

__global__ void __launch_bounds__(256)
k_so_sigma_fold(int n, const double *__restrict__ sig, const double *__restrict__ CSb, double *__restrict__ C2b) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n * n * n * n) return;
  C2b[e] += sig[(e / n) % n] * CSb[e];
}

// One workgroup of 256 per spatial (x, y): both spin blocks of the output,
// each a sum over the nonzero (same-spin) entries of D1 = diag(g, g), the
// threads striding over (spin of J, j, q); fixed-order reduction.
__global__ void __launch_bounds__(256)
k_so_d1bar_singlet(int r, const double *__restrict__ g, const double *__restrict__ cb, double *__restrict__ gb) {
  __shared__ double part[4];
  const int x = blockIdx.x / r, y = blockIdx.x % r;
  const int64_t n = 2 * (int64_t)r;
  auto at = [&](int64_t a, int64_t b, int64_t c, int64_t d) { return cb[((a * n + b) * n + c) * n + d]; };
  double acc = 0.0;
  const int64_t per = 2 * (int64_t)r * r;  // (spin of J, j, q)
  for (int sx = 0; sx < 2; ++sx) {
    const int64_t X = x + sx * r, Y = y + sx * r;
    for (int64_t e = threadIdx.x; e < per; e += 256) {
      const int q = (int)(e % r), j = (int)((e / r) % r), sj = (int)(e / ((int64_t)r * r));
      const int64_t J = j + sj * r, Q = q + sj * r;
      acc += g[j * r + q] * (at(X, J, Y, Q) + at(J, X, Q, Y) - at(J, X, Y, Q) - at(X, J, Q, Y));
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) gb[blockIdx.x] += -0.5 * (((part[0] + part[1]) + part[2]) + part[3]);
}

__global__ void __launch_bounds__(256)
k_spin_axpy(int64_t n, const double *x, double c, const double *__restrict__ y, double *out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) out[e] = x[e] + c * y[e];
}

inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

hipError_t launch_combine4(int r, const Terms4 &terms, double *out, int accumulate, const ActiveBits *mask,
                           hipStream_t s) {
  const int64_t n = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_combine4, grid1(n), dim3(256), 0, s, r, terms, out, accumulate, mask ? 1 : 0,
                     mask ? *mask : ActiveBits{});
  return hipGetLastError();
}

hipError_t launch_pack_op4(int r, const Terms4 &terms, double *out, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_op4, grid1((int64_t)r * r * ld), dim3(256), 0, s, r, terms, out, ld);
  return hipGetLastError();
}

hipError_t launch_outer4(int r, double c, const double *A, int a0, int a1, const double *B, int b0, int b1,
                         double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_outer4, grid1((int64_t)r * r * r * r), dim3(256), 0, s, r, c, A, a0, a1, B, b0, b1, out);
  return hipGetLastError();
}

hipError_t launch_trace12(int r, const double *in, double *out, int accumulate, hipStream_t s) {
  hipLaunchKernelGGL(k_trace12, grid1((int64_t)r * r), dim3(256), 0, s, r, in, out, accumulate);
  return hipGetLastError();
}

hipError_t launch_pair_traces(int r, int count, const double *const *in, double *traces, hipStream_t s) {
  TraceArgs a{};
  for (int q = 0; q < count && q < 8; ++q) a.in[q] = in[q];
  hipLaunchKernelGGL(k_pair_traces, dim3(count), dim3(256), 0, s, r, a, traces);
  return hipGetLastError();
}

hipError_t launch_spin_update(int r, double eps, double *const *d2, const double *const *U, const double *traces,
                              hipStream_t s) {
  UpdateArgs a{};
  for (int q = 0; q < 3; ++q) { a.d2[q] = d2[q]; a.U[q] = U[q]; }
  const int64_t n = (int64_t)r * r * r * r;
  hipLaunchKernelGGL(k_spin_update, dim3((unsigned)((n + 255) / 256), 3), dim3(256), 0, s, r, eps, a, traces);
  return hipGetLastError();
}

hipError_t launch_unpack_rows_lt(int r, const double *C, int64_t ldc, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_rows_lt, grid1((int64_t)r * r * r * r), dim3(256), 0, s, r, C, ldc, out);
  return hipGetLastError();
}

hipError_t launch_spin_axpy(int64_t n, const double *x, double c, const double *y, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_spin_axpy, grid1(n), dim3(256), 0, s, n, x, c, y, out);
  return hipGetLastError();
}

hipError_t launch_so_embed(int r, int bits, const double *in, double c, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_so_embed, grid1((int64_t)r * r * r * r), dim3(256), 0, s, r, bits, in, c, out);
  return hipGetLastError();
}

hipError_t launch_so_cumulant(int r, const double *ga, const double *gb, const double *d2aa, const double *d2bb,
                              const double *d2ab, const double *sig, double *c2, double *cs, hipStream_t s) {
  const int64_t n = 2 * (int64_t)r;
  hipLaunchKernelGGL(k_so_cumulant, grid1(n * n * n * n), dim3(256), 0, s, r, ga, gb, d2aa, d2bb, d2ab, sig, c2,
                     cs);
  return hipGetLastError();
}

hipError_t launch_so_trace_y(int n, const double *W, double *Y, hipStream_t s) {
  hipLaunchKernelGGL(k_so_trace_y, grid1((int64_t)n * n), dim3(256), 0, s, n, W, Y);
  return hipGetLastError();
}

hipError_t launch_so_tpl(int n, double c, const double *Y, const double *cs, double *B, hipStream_t s) {
  const int r = n / 2;
  if (r > kTplMaxR) return hipErrorInvalidValue;
  const size_t lds = 2 * (size_t)r * r * sizeof(double);
  hipLaunchKernelGGL(k_so_tpl, grid1((int64_t)n * n * n), dim3(256), lds, s, n, c, Y, cs, B);
  return hipGetLastError();
}

hipError_t launch_so_pack(int r, int64_t rpad, int64_t kc, const double *src, const int64_t st[4],
                          const int src_pos[4], int pair, double *out, hipStream_t s) {
  SoPackArgs a{};
  const int64_t ld = 4 * kc;
  // destination: row (2 s0 + s1) rpad + l0 r + l1, column (2 s2 + s3) kc + l2 r + l3
  const int64_t bb[4] = {(int64_t)r * ld, ld, r, 1};
  const int64_t oo[4] = {2 * rpad * ld, rpad * ld, 2 * kc, kc};
  for (int t = 0; t < 4; ++t) {
    a.st[t] = st[t];
    a.b[t] = bb[t];
    a.o[t] = oo[t];
    a.c[t] = (src_pos[t] == 0 || src_pos[t] == pair) ? 1 : -1;
  }
  a.u = 3;
  for (int t = 0; t < 3; ++t)
    if (st[t] == 1) a.u = t;
  // the fixed positions: the two of 0..2 other than u (for u = 3: positions 0 and 1)
  if (a.u == 3) { a.v = 0; a.w = 1; }
  else { a.v = a.u == 0 ? 1 : 0; a.w = a.u == 2 ? 1 : 2; }
  const int n = 2 * r;
  hipLaunchKernelGGL(k_so_pack, dim3((unsigned)((int64_t)n * n)), dim3(256), 0, s, r, src, a, out);
  return hipGetLastError();
}

hipError_t launch_so_embed_singlet_x(int r, const double *Aaa, const double *Aab, double *X, hipStream_t s) {
  const int64_t n = 2 * (int64_t)r;
  hipLaunchKernelGGL(k_so_embed_singlet_x, grid1(n * n * n * n), dim3(256), 0, s, r, Aaa, Aab, X);
  return hipGetLastError();
}

hipError_t launch_so_xbar_singlet(int r, const double *Xbar, double *Abaa, double *Abab, hipStream_t s) {
  hipLaunchKernelGGL(k_so_xbar_singlet, grid1((int64_t)r * r * r * r), dim3(256), 0, s, r, Xbar, Abaa, Abab);
  return hipGetLastError();
}

hipError_t launch_so_dbar_singlet(int r, double c, const double *D, double *Gaa, double *Gab, hipStream_t s) {
  hipLaunchKernelGGL(k_so_dbar_singlet, grid1((int64_t)r * r * r * r), dim3(256), 0, s, r, c, D, Gaa, Gab);
  return hipGetLastError();
}

hipError_t launch_so_bbar(int r, const double *Rbar_aa, const double *Rbar_ab, double sign, double *Bbar,
                          hipStream_t s) {
  const int64_t n = 2 * (int64_t)r;
  hipLaunchKernelGGL(k_so_bbar, grid1(n * n * n * n), dim3(256), 0, s, r, Rbar_aa, Rbar_ab, sign, Bbar);
  return hipGetLastError();
}

hipError_t launch_so_ybar(int n, double c, const double *Bbar, const double *cs, double *part, double *Ybar,
                          hipStream_t s) {
  const int r = n / 2;
  if (r > kTplMaxR) return hipErrorInvalidValue;
  const size_t lds = 2 * (size_t)r * (r + 1) * sizeof(double);
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_so_ybar_part),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(2 * (size_t)kTplMaxR * (kTplMaxR + 1) * sizeof(double)));
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_so_ybar_part, dim3(kSoYbarParts), dim3(256), lds, s, n, Bbar, cs, part);
  hipLaunchKernelGGL(k_so_ybar_sum, grid1((int64_t)n * n), dim3(256), 0, s, n, c, part, kSoYbarParts, Ybar);
  return hipGetLastError();
}

hipError_t launch_so_csbar_pl(int n, double c, const double *Bbar, const double *Y, double *CSbar, hipStream_t s) {
  const int r = n / 2;
  if (r > kTplMaxR) return hipErrorInvalidValue;
  const size_t lds = 2 * (size_t)r * r * sizeof(double);
  hipLaunchKernelGGL(k_so_csbar_pl, grid1((int64_t)n * n * n), dim3(256), lds, s, n, c, Bbar, Y, CSbar);
  return hipGetLastError();
}

hipError_t launch_so_diag_add(int n, const double *Ybar, double *Wbar, hipStream_t s) {
  hipLaunchKernelGGL(k_so_diag_add, grid1((int64_t)n * n * n), dim3(256), 0, s, n, Ybar, Wbar);
  return hipGetLastError();
}

hipError_t launch_so_sigma_fold(int n, const double *sig, const double *CSbar, double *C2bar, hipStream_t s) {
  hipLaunchKernelGGL(k_so_sigma_fold, grid1((int64_t)n * n * n * n), dim3(256), 0, s, n, sig, CSbar, C2bar);
  return hipGetLastError();
}

hipError_t launch_so_d1bar_singlet(int r, const double *g, const double *C2bar, double *gbar, hipStream_t s) {
  hipLaunchKernelGGL(k_so_d1bar_singlet, dim3((unsigned)(r * r)), dim3(256), 0, s, r, g, C2bar, gbar);
  return hipGetLastError();
}

hipError_t launch_spin_1rdm(int r, int N, const double *d2aa, const double *d2bb, const double *d2ab, double *ga,
                            double *gb, hipStream_t s) {
  hipLaunchKernelGGL(k_spin_1rdm, grid1((int64_t)r * r), dim3(256), 0, s, r, 2.0 / (N - 1), d2aa, d2bb, d2ab, ga,
                     gb);
  return hipGetLastError();
}

}  // namespace acse
