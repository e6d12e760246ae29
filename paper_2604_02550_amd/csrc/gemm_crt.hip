// Exact-accumulation products on the int8 MFMA: the pair-index products of
// the residual map in FP64 accuracy from integer matrix cores.
//
// Scheme (a modular, Chinese-remainder emulation of an FP64 product).  For
// C = A B^T with FP64 operands stored row by row over K:
//   1. every row of A and of B is scaled by a power of two to integers of at
//      most k bits:  A[m,:] ~ A_int[m,:] 2^(ea[m]-k),  |A_int| <= 2^k
//      (rounding to nearest; the only inexact step), likewise B;
//   2. the integers are reduced modulo pairwise coprime moduli m_j <= 256,
//      each residue in the int8 range; one operand carries the factor
//      u_j = (M/m_j)^-1 mod m_j (M = prod m_j);
//   3. one int8 MFMA product per modulus, accumulated exactly in int32
//      (|sum| <= K 128^2 < 2^31 for K < 131072);
//   4. y_j = acc_j mod m_j, and sum_j (M/m_j) y_j = A_int B_int^T (mod M);
//      with K 2^(2k) < M/4 the representative of smallest magnitude is the
//      exact integer product;
//   5. C = alpha * that integer * 2^(ea[m] + eb[n] - 2k), written through the
//      same 4-index store map as the floating-point products.
// The reconstruction runs in FP64: sum_j s1_j y_j is exact (s1_j = M/m_j with
// its low bits cleared, at most 41 significant bits), sum_j s2_j y_j carries
// the rest, and the multiple of M is removed from the exact part first.
//
// Kernel: 8 wavefronts (2 x 4) own a 128 x 128 tile, each wave 64 x 32 made
// of 16 x 16 blocks of v_mfma_i32_16x16x64_i8.  The loop runs over
// (modulus, K slab) pairs with double-buffered LDS slabs; after the last slab
// of a modulus the int32 accumulators are reduced and added to the two FP64
// reconstruction sums, then cleared.
#include <algorithm>
#include <cmath>

#include "gemm_crt.h"

namespace acse {

static_assert(sizeof(GemmBatch) + sizeof(CrtTable) <= 4096 - 64, "kernel arguments must fit in 4 KiB");
static_assert(sizeof(ResidueBatch) + sizeof(CrtTable) <= 4096 - 64, "kernel arguments must fit in 4 KiB");

namespace {

typedef int32_t v4i __attribute__((ext_vector_type(4)));

constexpr int kBM = 128, kBN = 128, kBK = 256;  // tile rows, columns, K bytes per slab
constexpr int kNT = 512;                        // 8 wavefronts
constexpr int kLDK = kBK + 16;                  // LDS row stride (bytes): 16 rows of a
                                                // 16-byte fragment read fall in distinct banks
constexpr int kGroupM = 8;

// XCD-aware logical workgroup index (the dispatcher deals workgroups round-robin
// over the 8 XCDs, each with its own L2): every XCD receives a contiguous range.
__device__ inline int xcd_logical_crt(int hw, int n) {
  const int xcd = hw % kGemmXcds, kx = hw / kGemmXcds;
  const int q8 = n / kGemmXcds, rem8 = n % kGemmXcds;
  return xcd < rem8 ? xcd * (q8 + 1) + kx : rem8 * (q8 + 1) + (xcd - rem8) * q8 + kx;
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

__device__ __forceinline__ void crt_tile(const GemmProb &P, const CrtTable &T, int local) {
  constexpr int WTM = kBM / 2, WTN = kBN / 4;  // 64 x 32 per wave
  constexpr int FM = WTM / 16, FN = WTN / 16;  // 4 x 2 MFMA blocks
  constexpr int NKK = kBK / 64;                // MFMA steps per slab
  constexpr int ROWB = kBK;                    // LDS row: 16 slots of 16 bytes, no padding
  constexpr int LPW = kBM * kBK / 1024 / (kNT / 64);  // 1 KB direct loads per wave per operand
  static_assert(kBK == 256, "the LDS swizzle assumes 16 slots of 16 bytes per row");
  static_assert(LPW * 1024 * (kNT / 64) == kBM * kBK, "tile must split into whole wave loads");
  static_assert(NKK >= 4 && NKK % 2 == 0, "pipelined loop needs an even step count >= 4");
  // LDS slot of logical 16-byte chunk c of row r: c ^ (r % 16).  The 16 rows a
  // fragment read takes (one chunk each) then fall on 16 distinct slots, i.e.
  // all 64 banks, and a direct load still fills 1 KB (4 rows) contiguously.
  __shared__ __attribute__((aligned(1024))) int8_t As[2][kBM * ROWB];
  __shared__ __attribute__((aligned(1024))) int8_t Bs[2][kBN * ROWB];

  // grouped tile order: kGroupM tile rows sweep the columns together
  const int in_group = kGroupM * P.tiles_n;
  const int group = local / in_group;
  const int first_m = group * kGroupM;
  const int gsz = min(P.tiles_m - first_m, kGroupM);
  const int lg = local - group * in_group;
  const int m0 = (first_m + lg % gsz) * kBM, n0 = (lg / gsz) * kBN;
  const int nk = P.Kp / kBK;
  const int nmod = T.nmod;
  const int total = nk * nmod;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 2) * WTM, wn0 = (wave & 3) * WTN;
  const int8_t *Ab = static_cast<const int8_t *>(P.A);
  const int8_t *Bb = static_cast<const int8_t *>(P.B);

  // Direct loads: load q of this wave fills LDS bytes [(wave LPW + q) KB, +1 KB)
  // = rows 16 wave + 4 q + lane / 16 (LPW = 4); lane l fetches the chunk that
  // belongs in slot l % 16 of its row, chunk (l % 16) ^ (row % 16) = c0 ^ 4q.
  static_assert(LPW == 4, "row r % 16 = 4 q + lane / 16 needs four loads per wave");
  const int c0 = (lane & 15) ^ (lane >> 4);
  const uint32_t ra0 = (uint32_t)((m0 + 16 * wave + (lane >> 4)) * P.ld);
  const uint32_t rb0 = (uint32_t)((n0 + 16 * wave + (lane >> 4)) * P.ld);
  const uint32_t ld4 = (uint32_t)(4 * P.ld);
  auto glds = [&](int it, int buf) {
    const int j = it / nk, kt = it - j * nk;
    const int8_t *a = Ab + j * P.plane_a + kt * kBK;
    const int8_t *b = Bb + j * P.plane_b + kt * kBK;
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
      const int lds_off = (wave * LPW + q) * 1024;
      const uint32_t col = (uint32_t)((c0 ^ (4 * q)) * 16) + q * ld4;
      __builtin_amdgcn_global_load_lds((gbl_void_t *)(a + ra0 + col), (lds_void_t *)(&As[buf][lds_off]), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gbl_void_t *)(b + rb0 + col), (lds_void_t *)(&Bs[buf][lds_off]), 16, 0, 0);
    }
  };

  v4i acc[FM][FN];
  double c1[FM][FN][4], c2[FM][FN][4];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc[i][j] = v4i{0, 0, 0, 0};
#pragma unroll
      for (int v = 0; v < 4; ++v) { c1[i][j][v] = 0.0; c2[i][j][v] = 0.0; }
    }

  const int lrow = lane & 15;
  const int lgrp = lane >> 4;
  v4i fa[2][FM], fb[2][FN];
  auto fread = [&](int q, int b, int step) {
    const int slot = ((step * 4 + lgrp) ^ lrow) * 16;  // rows of a fragment are 16-aligned
#pragma unroll
    for (int i = 0; i < FM; ++i)
      fa[q][i] = *reinterpret_cast<const v4i *>(&As[b][(wm0 + i * 16 + lrow) * ROWB + slot]);
#pragma unroll
    for (int j = 0; j < FN; ++j)
      fb[q][j] = *reinterpret_cast<const v4i *>(&Bs[b][(wn0 + j * 16 + lrow) * ROWB + slot]);
  };
  auto mma = [&](int q) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[q][i], fb[q][j], acc[i][j], 0, 0, 0);
  };

  // Software-pipelined slab loop: the fragments of two MFMA steps are in
  // registers or in flight; the last two steps of a slab read the first two of
  // the next slab.  One barrier per slab, before the last step: after it every
  // wave's direct loads of the next slab have landed and every read of this
  // slab has completed, so the loads of the slab after next go into this
  // slab's buffer right away (they have about one slab of MFMAs to arrive).
  // Past the last slab the loads repeat the last one into the free buffer.
  glds(0, 0);
  glds(min(1, total - 1), 1);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  fread(0, 0, 0);
  __builtin_amdgcn_sched_barrier(0);
  fread(1, 0, 1);
  __builtin_amdgcn_sched_barrier(0);
  int it = 0;
  for (int j = 0; j < nmod; ++j) {
    for (int kt = 0; kt < nk; ++kt, ++it) {
      const int cur = it & 1;
#pragma unroll
      for (int s = 0; s < NKK; ++s) {
        mma(s & 1);
        __builtin_amdgcn_sched_barrier(0);
        if (s + 2 < NKK) {
          fread(s & 1, cur, s + 2);
        } else {
          if (s == NKK - 2) {
            __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the next slab
            __syncthreads();
            glds(min(it + 2, total - 1), cur);
          }
          fread(s & 1, cur ^ 1, s + 2 - NKK);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // modulus j complete.  Any y = acc (mod m) with |y| <= 128 keeps the
    // exact part of the reconstruction exact (41 + 7 bits per term, at most 15
    // terms), so y = acc - m rint(acc / m) needs no range correction.
    const double m = T.m[j], inv_m = T.inv_m[j], s1 = T.s1[j], s2 = T.s2[j];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int jj = 0; jj < FN; ++jj) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double a = (double)acc[i][jj][v];
          const double y = fma(-rint(a * inv_m), m, a);
          c1[i][jj][v] = fma(s1, y, c1[i][jj][v]);
          c2[i][jj][v] = fma(s2, y, c2[i][jj][v]);
        }
        acc[i][jj] = v4i{0, 0, 0, 0};
      }
  }

  // --- epilogue: integer product, scaling, (m, n) -> permuted 4-index address
  const double alpha = P.alpha;
  double *C = P.C;
  const int rdiv = P.rdiv;
  const double M1 = T.M1, M2 = T.M2, inv_M = T.inv_M;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn0 + j * 16 + lrow;
      if (n >= P.N) continue;
      const int64_t noff = (int64_t)(n / rdiv) * P.sn1 + (int64_t)(n % rdiv) * P.sn0;
      const int en = P.eb[n] - P.kshift;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // accumulator item v of lane l is row 4 (l / 16) + v, column l % 16
        const int m = m0 + wm0 + i * 16 + (lane >> 4) * 4 + v;
        if (m >= P.M) continue;
        const double q = rint((c1[i][j][v] + c2[i][j][v]) * inv_M);
        const double cint = fma(-q, M1, c1[i][j][v]) + fma(-q, M2, c2[i][j][v]);
        const double val = alpha * ldexp(cint, P.ea[m] + en);
        const int64_t off = (int64_t)(m / rdiv) * P.sm1 + (int64_t)(m % rdiv) * P.sm0 + noff;
        if (P.accumulate) C[off] += val; else C[off] = val;
      }
    }
  }
}

__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(2)))
gemm_crt_kernel(const GemmBatch batch, const CrtTable tab) {
  const int bid = xcd_logical_crt(blockIdx.x, batch.total_tiles);
  int lo = 0, hi = batch.nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (batch.seg_start[mid] <= bid) lo = mid; else hi = mid - 1;
  }
  crt_tile(batch.p[batch.seg_prob[lo]], tab, batch.seg_local[lo] + bid - batch.seg_start[lo]);
}

// ---------------------------------------------------------------------------
// Operand conversion: FP64 rows -> per-row exponent and int8 residue planes.
// One block per row: the row is staged in LDS, its largest magnitude gives the
// exponent e (|x| < 2^e), every element becomes the integer a = rint(x 2^(k-e))
// (|a| <= 2^k <= 2^50, exact in FP64) and its residue modulo each m_j in the
// int8 range (times u_j for the operand that carries the reconstruction
// factors).  Columns from K to the residue row stride are written as zero.
//
// Residues: for odd m, a - m rint(a / m) is exact and lies in [-(m-1)/2,
// (m-1)/2] (a / m is never within 1/(2m) of a half-integer, and for
// |a| <= 2^50 the rounding error of a (1/m) stays below 1/(4m)); for m = 256 the
// residue in [-128, 127] is the low byte of a mod 256 read as a signed byte.
// ---------------------------------------------------------------------------
__device__ inline int res_odd(double a, double m, double inv_m) { return (int)fma(-rint(a * inv_m), m, a); }

__device__ inline uint32_t pack4(int r0, int r1, int r2, int r3) {
  return (uint32_t)(r0 & 255) | ((uint32_t)(r1 & 255) << 8) | ((uint32_t)(r2 & 255) << 16) |
         ((uint32_t)(r3 & 255) << 24);
}

__global__ void __launch_bounds__(256) k_to_residues(const ResidueBatch b, const CrtTable T) {
  extern __shared__ double res_row[];
  __shared__ double wmax[4];
  int q = 0;
  while (q + 1 < b.count && b.job[q + 1].row_begin <= (int)blockIdx.x) ++q;
  const ResidueJob &J = b.job[q];
  const int row = blockIdx.x - J.row_begin;
  const int tid = threadIdx.x;
  const double *src = J.src + (int64_t)row * J.ld;
  double mx = 0.0;
  for (int k = tid; k < J.K; k += 256) {
    const double x = src[k];
    res_row[k] = x;
    mx = fmax(mx, fabs(x));
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if ((tid & 63) == 0) wmax[tid >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
  int e = 0;
  if (mx > 0.0) (void)frexp(mx, &e);  // mx = f 2^e, 0.5 <= f < 1
  if (tid == 0) J.e[row] = e;
  const double scale = ldexp(1.0, J.kbits - e);
  int8_t *dst = J.dst + (int64_t)row * J.ldr;
  const int nmod = T.nmod;
  for (int g = tid; g < J.ldr / 4; g += 256) {
    double a[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int k = 4 * g + t;
      a[t] = k < J.K ? rint(res_row[k] * scale) : 0.0;
    }
    // modulus 0 is 256: a mod 256 in [0, 256) (exact), stored as its low byte
    // (times u_0 for the factor-carrying side; the product stays below 2^16)
    {
      int r[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        r[t] = (int)fma(-floor(a[t] * (1.0 / 256.0)), 256.0, a[t]);
        if (J.premul) r[t] *= T.u[0];
      }
      *reinterpret_cast<uint32_t *>(dst + 4 * g) = pack4(r[0], r[1], r[2], r[3]);
    }
    for (int j = 1; j < nmod; ++j) {
      const double m = T.m[j], inv_m = T.inv_m[j];
      int r[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        r[t] = res_odd(a[t], m, inv_m);
        if (J.premul) r[t] = res_odd((double)(r[t] * T.u[j]), m, inv_m);
      }
      *reinterpret_cast<uint32_t *>(dst + j * J.plane + 4 * g) = pack4(r[0], r[1], r[2], r[3]);
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {
// pairwise coprime moduli <= 256, largest first
constexpr int kModuli[kMaxModuli] = {256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197};

using u128 = unsigned __int128;
int bitlen(u128 x) {
  int n = 0;
  while (x) { ++n; x >>= 1; }
  return n;
}
double u128_to_double(u128 x) {
  return (double)(uint64_t)(x >> 64) * 18446744073709551616.0 + (double)(uint64_t)x;
}
int64_t inv_mod(int64_t a, int64_t m) {  // a^-1 mod m (a, m coprime)
  int64_t t = 0, nt = 1, r = m, nr = ((a % m) + m) % m;
  while (nr) {
    const int64_t qq = r / nr;
    int64_t tmp = t - qq * nt; t = nt; nt = tmp;
    tmp = r - qq * nr; r = nr; nr = tmp;
  }
  return ((t % m) + m) % m;
}
}  // namespace

bool crt_table(int nmod, CrtTable &T) {
  static_assert(kModuli[0] == 256, "the residue kernel takes modulus 0 as 256 (low bytes)");
  if (nmod < kMinModuli || nmod > kMaxModuli) return false;
  T = CrtTable{};
  T.nmod = nmod;
  u128 M = 1;
  double log2M = 0.0;
  for (int j = 0; j < nmod; ++j) {
    M *= (u128)kModuli[j];
    log2M += std::log2((double)kModuli[j]);
  }
  T.log2M = log2M;
  u128 smax = 0;
  for (int j = 0; j < nmod; ++j) smax = std::max(smax, M / (u128)kModuli[j]);
  const int t = std::max(0, bitlen(smax) - 41);  // s1_j: at most 41 significant bits
  for (int j = 0; j < nmod; ++j) {
    const int m = kModuli[j];
    const u128 s = M / (u128)m;
    const u128 s1 = (s >> t) << t;
    T.m[j] = m;
    T.inv_m[j] = 1.0 / m;
    T.s1[j] = u128_to_double(s1);                 // exact
    T.s2[j] = u128_to_double(s - s1);             // rounded
    T.u[j] = (int)inv_mod((int64_t)(s % (u128)m), m);
  }
  const int tm = std::max(0, bitlen(M) - 40);      // q M1 exact for |q| < 2^12
  const u128 M1 = (M >> tm) << tm;
  T.M1 = u128_to_double(M1);
  T.M2 = u128_to_double(M - M1);
  T.inv_M = 1.0 / u128_to_double(M);
  return true;
}

int crt_kbits(const CrtTable &T, int K) {
  // K 2^(2k) < M / 4  <=>  2k < log2 M - log2 K - 2.  At most 50 bits: for
  // |a| <= 2^50 the error of a (1/m) stays below a quarter of 1/m, so rint(a / m)
  // is exact for the odd moduli (the residue kernel relies on it).
  const double room = T.log2M - std::log2((double)std::max(K, 1)) - 2.0;
  int k = (int)std::floor(room / 2.0);
  while (k > 0 && 2.0 * k >= room) --k;
  return std::min(k, 50);
}

int64_t crt_ldr(int K) { return round_up(std::max(K, 1), kCrtKPad); }

hipError_t launch_to_residues(const ResidueBatch &b, const CrtTable &T, hipStream_t s) {
  if (b.total_rows == 0) return hipSuccess;
  int kmax = 1;
  for (int q = 0; q < b.count; ++q) kmax = std::max(kmax, b.job[q].K);
  const size_t lds = (size_t)kmax * sizeof(double);  // one staged row (74 KB at K = 96^2)
  if (lds > 48 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_to_residues),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_to_residues, dim3(b.total_rows), dim3(256), lds, s, b, T);
  return hipGetLastError();
}

hipError_t gemm_crt_launch(GemmBatch &b, const CrtTable &T, hipStream_t s) {
  int total = 0;
  for (int q = 0; q < b.count; ++q) {
    GemmProb &p = b.p[q];
    p.tiles_m = (p.M + kBM - 1) / kBM;
    p.tiles_n = (p.N + kBN - 1) / kBN;
    p.ksplit = 1;
    p.kchunk = p.Kp;
    p.tile_begin = total;
    total += p.tiles_m * p.tiles_n;
  }
  b.total_tiles = total;
  if (total == 0) return hipSuccess;
  // each XCD's contiguous range holds an equal share of every problem
  b.nseg = 0;
  int start = 0;
  for (int c = 0; c < kGemmXcds; ++c)
    for (int q = 0; q < b.count; ++q) {
      const int n = b.p[q].tiles_m * b.p[q].tiles_n;
      const int lo = (int)((int64_t)n * c / kGemmXcds), hi = (int)((int64_t)n * (c + 1) / kGemmXcds);
      if (hi <= lo) continue;
      b.seg_start[b.nseg] = start;
      b.seg_prob[b.nseg] = q;
      b.seg_local[b.nseg] = lo;
      ++b.nseg;
      start += hi - lo;
    }
  b.seg_start[b.nseg] = start;
  hipLaunchKernelGGL(gemm_crt_kernel, dim3(total), dim3(kNT), 0, s, b, T);
  return hipGetLastError();
}

}  // namespace acse
