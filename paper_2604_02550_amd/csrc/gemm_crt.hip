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
//      u_j = (M/m_j)^-1 mod m_j (M = prod m_j), or (u_out) the product's
//      residues are multiplied by it;
//   3. one int8 MFMA product per modulus, accumulated exactly in int32
//      (|sum| <= K 128^2 < 2^31 for K < 131072), reduced to a residue
//      y_j = acc_j mod m_j (times u_j with u_out) in the int8 range and stored;
//   4. sum_j (M/m_j) y_j = A_int B_int^T (mod M); with K 2^(2k) < M/4 the
//      representative of smallest magnitude is the exact integer product;
//   5. C = alpha * that integer * 2^(ea[m] + eb[n] - 2k), written through the
//      same 4-index store map as the floating-point products.
// The reconstruction runs in FP64: sum_j s1_j y_j is exact (s1_j = M/m_j with
// its low bits cleared, at most 41 significant bits, |y_j| <= 128), sum_j
// s2_j y_j carries the rest, and the multiple of M is removed from the exact
// part first.
//
// Kernels: the residue conversion of the operands (one block per row), the
// modular product (256 x 256 tiles, one modulus per tile; 8 wavefronts of
// 128 x 64 on v_mfma_i32_32x32x32_i8; K slabs loaded straight into LDS) and
// the reconstruction (one thread per four rows of one column).
#include <algorithm>
#include <cmath>
#include <vector>

#include "gemm_crt.h"

namespace acse {

static_assert(sizeof(GemmBatch) + sizeof(CrtTable) + sizeof(ModSched) <= 4096 - 64, "kernel arguments must fit in 4 KiB");
static_assert(sizeof(ResidueBatch) + sizeof(CrtTable) <= 4096 - 64, "kernel arguments must fit in 4 KiB");

namespace {

typedef int32_t v4i __attribute__((ext_vector_type(4)));

constexpr int kBM = 256, kBN = 256, kBK = 128;  // tile rows, columns, K bytes per slab
constexpr int kNT = 512;                        // 8 wavefronts
constexpr int kGroupM = 8;

typedef int32_t v16i __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

// One 256 x 256 tile of one product for one modulus: C_j = A_j B_j^T, reduced
// to residues y = C_j mod m_j in [-128, 128] (stored as bytes; y = 128 only
// for m = 256, where the byte -128 is the same residue).
__device__ __forceinline__ void mod_tile(const GemmProb &P, const CrtTable &T, int j, int local) {
  constexpr int WTM = kBM / 2, WTN = kBN / 4;  // 128 x 64 per wave
  constexpr int FM = WTM / 32, FN = WTN / 32;  // 4 x 2 blocks of 32 x 32
  constexpr int NKK = kBK / 32;                // MFMA steps per slab
  constexpr int ROWB = kBK;                    // LDS row: 8 slots of 16 bytes, no padding
  constexpr int LPW = kBM * kBK / 1024 / (kNT / 64);  // 1 KB direct loads per wave per operand
  static_assert(kBK == 128 && LPW == 4, "the LDS swizzle and load mapping assume 128-byte rows");
  static_assert(NKK >= 4 && NKK % 2 == 0, "pipelined loop needs an even step count >= 4");
  // LDS slot of logical 16-byte chunk c of row r: c ^ ((r / 2) % 8).  The 16
  // rows a quarter-wave of a fragment read takes (same chunk) then cover all
  // 64 banks once (two rows share a 256-byte bank line), and a direct load
  // still fills 1 KB (8 rows) contiguously.
  // Two stages of A and B, each its own array: the loads of one stage and the
  // fragment reads of the other then provably touch different LDS objects,
  // so no wait for the loads in flight is inserted before those reads.
  __shared__ __attribute__((aligned(1024))) int8_t As0[kBM * ROWB];
  __shared__ __attribute__((aligned(1024))) int8_t As1[kBM * ROWB];
  __shared__ __attribute__((aligned(1024))) int8_t Bs0[kBN * ROWB];
  __shared__ __attribute__((aligned(1024))) int8_t Bs1[kBN * ROWB];

  // grouped tile order: kGroupM tile rows sweep the columns together
  const int in_group = kGroupM * P.tiles_n;
  const int group = local / in_group;
  const int first_m = group * kGroupM;
  const int gsz = min(P.tiles_m - first_m, kGroupM);
  const int lg = local - group * in_group;
  const int m0 = (first_m + lg % gsz) * kBM, n0 = (lg / gsz) * kBN;
  const int nk = P.Kp / kBK;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 2) * WTM, wn0 = (wave & 3) * WTN;
  const int8_t *Ab = static_cast<const int8_t *>(P.A) + j * P.plane_a;
  const int8_t *Bb = static_cast<const int8_t *>(P.B) + j * P.plane_b;

  // Direct loads: load q of this wave fills LDS bytes [(wave LPW + q) KB, +1 KB)
  // = rows 32 wave + 8 q + lane / 8; lane l fetches the chunk that belongs in
  // slot l % 8 of its row: chunk (l % 8) ^ ((row / 2) % 8) = (l % 8) ^ ((4 q + l / 16) % 8).
  const uint32_t ra0 = (uint32_t)((m0 + 32 * wave + (lane >> 3)) * P.ld);
  const uint32_t rb0 = (uint32_t)((n0 + 32 * wave + (lane >> 3)) * P.ld);
  const uint32_t ld8 = (uint32_t)(8 * P.ld);
  auto glds = [&](int kt, int8_t *as, int8_t *bs) {
    const int8_t *a = Ab + kt * kBK;
    const int8_t *b = Bb + kt * kBK;
#pragma unroll
    for (int q = 0; q < LPW; ++q) {
      const int lds_off = (wave * LPW + q) * 1024;
      const uint32_t col = (uint32_t)(((lane & 7) ^ ((4 * q + (lane >> 4)) & 7)) * 16) + q * ld8;
      __builtin_amdgcn_global_load_lds((gbl_void_t *)(a + ra0 + col), (lds_void_t *)(as + lds_off), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((gbl_void_t *)(b + rb0 + col), (lds_void_t *)(bs + lds_off), 16, 0, 0);
    }
  };

  v16i acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int jj = 0; jj < FN; ++jj)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][jj][v] = 0;

  // fragment reads: lane l takes row (block base + l % 32), chunk 2 step + l / 32
  const int lrow = lane & 31;
  const int lhalf = lane >> 5;
  const int swz = (lrow >> 1) & 7;  // block bases are multiples of 32
  v4i fa[2][FM], fb[2][FN];
  auto fread = [&](int q, const int8_t *as, const int8_t *bs, int step) {
    const int slot = ((2 * step + lhalf) ^ swz) * 16;
#pragma unroll
    for (int i = 0; i < FM; ++i)
      fa[q][i] = *reinterpret_cast<const v4i *>(as + (wm0 + i * 32 + lrow) * ROWB + slot);
#pragma unroll
    for (int jj = 0; jj < FN; ++jj)
      fb[q][jj] = *reinterpret_cast<const v4i *>(bs + (wn0 + jj * 32 + lrow) * ROWB + slot);
  };
  auto mma = [&](int q) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int jj = 0; jj < FN; ++jj)
        acc[i][jj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[q][i], fb[q][jj], acc[i][jj], 0, 0, 0);
  };

  // Software-pipelined slab loop: the fragments of two MFMA steps are in
  // registers or in flight; the last two steps of a slab read the first two of
  // the next slab.  One barrier per slab, before the last step: after it every
  // wave's direct loads of the next slab have landed and every read of this
  // slab has completed, so the loads of the slab after next go into this
  // slab's buffer right away.  Past the last slab the loads repeat the last one.
  // One slab from stage (ac, bc); the next one is in (an, bn).
  auto slab = [&](int kt, int8_t *ac, int8_t *bc, int8_t *an, int8_t *bn) {
#pragma unroll
    for (int s = 0; s < NKK; ++s) {
      mma(s & 1);
      __builtin_amdgcn_sched_barrier(0);
      if (s + 2 < NKK) {
        fread(s & 1, ac, bc, s + 2);
      } else {
        if (s == NKK - 2) {
          __builtin_amdgcn_s_waitcnt(0);  // this wave's loads of the next slab
          __syncthreads();
          glds(min(kt + 2, nk - 1), ac, bc);
        }
        fread(s & 1, an, bn, s + 2 - NKK);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  glds(0, As0, Bs0);
  glds(min(1, nk - 1), As1, Bs1);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  fread(0, As0, Bs0, 0);
  __builtin_amdgcn_sched_barrier(0);
  fread(1, As0, Bs0, 1);
  __builtin_amdgcn_sched_barrier(0);
  int kt = 0;
  for (; kt + 1 < nk; kt += 2) {
    slab(kt, As0, Bs0, As1, Bs1);
    slab(kt + 1, As1, Bs1, As0, Bs0);
  }
  if (kt < nk) slab(kt, As0, Bs0, As1, Bs1);

  // residues, four consecutive rows of one column per 32-bit store:
  // accumulator item v of lane l is row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32
  const double m = T.m[j], inv_m = T.inv_m[j];
  const int um = T.u[j];
  int8_t *Y = P.Y + j * P.plane_y;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int jj = 0; jj < FN; ++jj) {
      const int n = n0 + wn0 + jj * 32 + lrow;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int row = m0 + wm0 + i * 32 + 8 * g + 4 * lhalf;
        uint32_t w = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double a = (double)acc[i][jj][4 * g + t];
          int y = (int)fma(-rint(a * inv_m), m, a);
          if (P.u_out) {  // |y u| < 2^15: exact
            const double yu = (double)(y * um);
            y = (int)fma(-rint(yu * inv_m), m, yu);
          }
          w |= (uint32_t)(y & 255) << (8 * t);
        }
        if (row < P.M && n < P.N) *reinterpret_cast<uint32_t *>(Y + ((int64_t)(row >> 2) * P.N + n) * 4) = w;
      }
    }
}

// Work of the modular product: every (product, modulus) pair runs whole on
// one XCD (own L2), so the tiles that XCD's CUs hold at one time are a compact
// block of one product and share their operand panels in its L2.  Workgroups
// go to XCDs round-robin by index (blockIdx.x % 8), and each XCD starts its
// workgroups in index order.
__global__ void __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(2)))
gemm_mod_kernel(const GemmBatch batch, const CrtTable tab, const ModSched sched) {
  const int c = blockIdx.x % kGemmXcds, s = blockIdx.x / kGemmXcds;
  int lo = sched.xs[c], hi = sched.xs[c + 1] - 1;
  if (hi < lo || s < sched.start[lo]) return;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sched.start[mid] <= s) lo = mid; else hi = mid - 1;
  }
  const GemmProb &P = batch.p[sched.prob[lo]];
  const int local = s - sched.start[lo];
  if (local >= P.tiles_m * P.tiles_n) return;
  mod_tile(P, tab, sched.mod[lo], local);
}

// Reconstruction: one thread per (product, row quad, column).
__global__ void __launch_bounds__(256) k_crt_combine(const GemmBatch batch, const CrtTable T) {
  const GemmProb &P = batch.p[blockIdx.y];
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nquad = (P.M + 3) / 4;
  if (idx >= nquad * P.N) return;
  const int q = (int)(idx / P.N), n = (int)(idx - (int64_t)q * P.N);
  double c1[4] = {0.0, 0.0, 0.0, 0.0}, c2[4] = {0.0, 0.0, 0.0, 0.0};
  const int8_t *Y = P.Y + idx * 4;
  // every modulus' word in flight at once, then the sums
  uint32_t w[kMaxModuli];
#pragma unroll
  for (int j = 0; j < kMaxModuli; ++j)
    w[j] = j < T.nmod ? *reinterpret_cast<const uint32_t *>(Y + j * P.plane_y) : 0u;
#pragma unroll
  for (int j = 0; j < kMaxModuli; ++j) {
    const double s1 = T.s1[j], s2 = T.s2[j];  // zero beyond nmod
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double y = (double)(int8_t)(w[j] >> (8 * t));
      c1[t] = fma(s1, y, c1[t]);
      c2[t] = fma(s2, y, c2[t]);
    }
  }
  const int en = P.eb[n] - P.kshift;
  const int64_t noff = (int64_t)(n / P.rdiv) * P.sn1 + (int64_t)(n % P.rdiv) * P.sn0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int m = 4 * q + t;
    if (m >= P.M) break;
    const double qq = rint((c1[t] + c2[t]) * T.inv_M);
    const double cint = fma(-qq, T.M1, c1[t]) + fma(-qq, T.M2, c2[t]);
    const double val = P.alpha * ldexp(cint, P.ea[m] + en);
    const int64_t off = (int64_t)(m / P.rdiv) * P.sm1 + (int64_t)(m % P.rdiv) * P.sm0 + noff;
    if (P.accumulate) P.C[off] += val; else P.C[off] = val;
  }
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
  // four loads in flight per thread
  int k0 = tid;
  for (; k0 + 3 * 256 < J.K; k0 += 4 * 256) {
    double x[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) x[t] = src[k0 + t * 256];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      res_row[k0 + t * 256] = x[t];
      mx = fmax(mx, fabs(x[t]));
    }
  }
  for (; k0 < J.K; k0 += 256) {
    const double x = src[k0];
    res_row[k0] = x;
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
  // Longest-first assignment of the (product, modulus) pairs to XCDs by cost
  // (tiles x K slabs), then each XCD's pairs in modulus order, so that the XCDs
  // work on few moduli at a time and the Infinity Cache holds their planes.
  if (b.count * T.nmod > kMaxModPairs) return hipErrorInvalidValue;
  struct Pair { int q, j; int64_t cost; };
  std::vector<Pair> pairs;
  for (int j = 0; j < T.nmod; ++j)
    for (int q = 0; q < b.count; ++q) {
      const GemmProb &p = b.p[q];
      const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
      if (tiles > 0) pairs.push_back({q, j, tiles * (p.Kp / kBK)});
    }
  std::vector<int> order(pairs.size());
  for (size_t e = 0; e < order.size(); ++e) order[e] = (int)e;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return pairs[x].cost > pairs[y].cost; });
  int64_t load[kGemmXcds] = {};
  std::vector<int> owner(pairs.size());
  for (int e : order) {
    int best = 0;
    for (int c = 1; c < kGemmXcds; ++c)
      if (load[c] < load[best]) best = c;
    owner[e] = best;
    load[best] += pairs[e].cost;
  }
  ModSched sched{};
  int n = 0, share = 0;
  for (int c = 0; c < kGemmXcds; ++c) {
    sched.xs[c] = n;
    int t = 0;
    for (size_t e = 0; e < pairs.size(); ++e) {  // pairs are listed modulus-major
      if (owner[e] != c) continue;
      sched.start[n] = t;
      sched.prob[n] = (uint8_t)pairs[e].q;
      sched.mod[n] = (uint8_t)pairs[e].j;
      t += b.p[pairs[e].q].tiles_m * b.p[pairs[e].q].tiles_n;
      ++n;
    }
    share = std::max(share, t);
  }
  sched.xs[kGemmXcds] = n;
  b.nseg = 0;
  hipLaunchKernelGGL(gemm_mod_kernel, dim3(kGemmXcds * share), dim3(kNT), 0, s, b, T, sched);
  return hipGetLastError();
}

hipError_t crt_combine_launch(const GemmBatch &b, const CrtTable &T, hipStream_t s) {
  if (b.total_tiles == 0) return hipSuccess;
  int64_t most = 0;
  for (int q = 0; q < b.count; ++q) most = std::max(most, (int64_t)((b.p[q].M + 3) / 4) * b.p[q].N);
  hipLaunchKernelGGL(k_crt_combine, dim3((unsigned)((most + 255) / 256), b.count), dim3(256), 0, s, b, T);
  return hipGetLastError();
}

int64_t crt_residue_out_bytes(int M, int N) { return (int64_t)round_up(M, 4) * N; }

}  // namespace acse
