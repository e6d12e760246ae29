// LDS-tiled MFMA NT GEMMs for gfx950 (FP64, FP32, split-BF16).
//
// Every O(r^6) contraction of the residual is a pair-index product
// C[(a,b),(c,d)] = sum_(e,f) A[(a,b),(e,f)] B[(c,d),(e,f)] with r^2 x r^2
// operands; this file holds the one kernel that runs them all.
//
// Structure: a workgroup of 4 wavefronts (2 x 2) owns a BM x BN output tile;
// each wave owns a (BM/2) x (BN/2) sub-tile made of 16 x 16 MFMA blocks.  The
// K loop stages BK-wide slabs of A and B through LDS with register
// double-buffering (the next slab's global loads are in flight while the
// current slab feeds the MFMAs).  LDS rows are padded so that the 16 rows a
// half-wave reads for one MFMA operand fall in distinct banks.
#include <algorithm>
#include <vector>

#include "acse_internal.h"

namespace acse {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// PAD: LDS row padding in elements.  Fragment reads take one element per lane
// from 16 consecutive rows (and 4 consecutive k).  FP64: a 64-bit read serves
// 32 lanes (16 rows x 2 k) per pass, and a row stride of BK + 2 doubles puts
// them on 32 distinct bank pairs (BK + 1 leaves one 2-way conflict per pass);
// the rows also stay 16-byte aligned for whole-chunk staging stores.  FP32: a
// row stride of BK + 4 floats keeps the rows 16-byte aligned (whole-chunk
// stores); the counters still show some conflicts on its 32-bit reads, with
// the same product time as the odd stride BK + 1.
struct TrF64 {
  using T = double;
  using Acc = d4;
  static constexpr int NPLANE = 1, VEC = 2, PAD = 2, KSTEP = 4;
};
struct TrF32 {
  using T = float;
  using Acc = f4;
  static constexpr int NPLANE = 1, VEC = 4, PAD = 4, KSTEP = 4;
};
struct TrBF16x3 {
  using T = __bf16;
  using Acc = f4;
  static constexpr int NPLANE = 2, VEC = 8, PAD = 8, KSTEP = 32;
};

template <class Tr>
__device__ inline typename Tr::Acc acc_zero() {
  typename Tr::Acc a;
  a[0] = 0; a[1] = 0; a[2] = 0; a[3] = 0;
  return a;
}

constexpr int kNumXcd = kGemmXcds;
constexpr int kGroupM = 8;

// One BM x BN output tile (and K chunk) of problem P; `local` counts the
// problem's tiles in grouped order (split-major).  NS = 2: double-buffered LDS
// slabs (one barrier per slab); NS = 1: one LDS slab (half the LDS, so twice
// the resident workgroups for wide slabs), refilled from the register prefetch
// between two barriers.
template <class Tr, int BM, int BN, int BK, int NS>
__device__ __forceinline__ void gemm_tile(const GemmProb &P, int local) {
  using T = typename Tr::T;
  using Acc = typename Tr::Acc;
  constexpr int NT = 256;
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  constexpr int LDK = BK + Tr::PAD;
  constexpr int NP = Tr::NPLANE;
  constexpr int VEC = Tr::VEC;
  constexpr int CH_A = BM * BK / VEC / NT;   // 16-byte chunks per thread per plane
  constexpr int CH_B = BN * BK / VEC / NT;
  static_assert(CH_A * VEC * NT == BM * BK, "A tile must split evenly");
  static_assert(CH_B * VEC * NT == BN * BK, "B tile must split evenly");
  static_assert(BK % Tr::KSTEP == 0, "K tile must hold whole MFMA steps");

  __shared__ __attribute__((aligned(16))) T As[NS][NP][BM * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[NS][NP][BN * LDK];

  // --- which tile / K chunk --------------------------------------------------
  const int per_split = P.tiles_m * P.tiles_n;
  const int split = local / per_split;
  local -= split * per_split;
  // grouped order: kGroupM tile rows sweep the columns together so the
  // resident workgroups share A and B panel slabs in L2
  const int in_group = kGroupM * P.tiles_n;
  const int group = local / in_group;
  const int first_m = group * kGroupM;
  const int gsz = min(P.tiles_m - first_m, kGroupM);
  const int lg = local - group * in_group;
  const int tm = first_m + lg % gsz;
  const int tn = lg / gsz;
  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = split * P.kchunk;
  const int kend = min(P.Kp, kbeg + P.kchunk);
  const int nk = (kend - kbeg) / BK;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * WTM, wn0 = (wave & 1) * WTN;

  const T *Ap[2] = {static_cast<const T *>(P.A), static_cast<const T *>(NP > 1 ? P.A2 : P.A)};
  const T *Bp[2] = {static_cast<const T *>(P.B), static_cast<const T *>(NP > 1 ? P.B2 : P.B)};
  const int64_t ld = P.ld;

  // 16-byte global chunks -> registers
  typedef int32_t i4 __attribute__((ext_vector_type(4)));
  i4 ra[NP][CH_A], rb[NP][CH_B];
  auto gload = [&](int k0) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int c = 0; c < CH_A; ++c) {
        const int ch = tid + c * NT;
        const int row = ch / (BK / VEC), kc = (ch % (BK / VEC)) * VEC;
        ra[p][c] = *reinterpret_cast<const i4 *>(Ap[p] + (int64_t)(m0 + row) * ld + k0 + kc);
      }
#pragma unroll
      for (int c = 0; c < CH_B; ++c) {
        const int ch = tid + c * NT;
        const int row = ch / (BK / VEC), kc = (ch % (BK / VEC)) * VEC;
        rb[p][c] = *reinterpret_cast<const i4 *>(Bp[p] + (int64_t)(n0 + row) * ld + k0 + kc);
      }
    }
  };
  // 16-byte chunk -> LDS at element offset o (whole-chunk store when the row
  // stride keeps chunks 16-byte aligned, element stores otherwise)
  auto put16 = [&](T *base, int o, const i4 &v) {
    if constexpr ((LDK * sizeof(T)) % 16 == 0) {
      *reinterpret_cast<i4 *>(base + o) = v;
    } else {
      const T *e = reinterpret_cast<const T *>(&v);
#pragma unroll
      for (int q = 0; q < VEC; ++q) base[o + q] = e[q];
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int c = 0; c < CH_A; ++c) {
        const int ch = tid + c * NT;
        const int row = ch / (BK / VEC), kc = (ch % (BK / VEC)) * VEC;
        put16(As[buf][p], row * LDK + kc, ra[p][c]);
      }
#pragma unroll
      for (int c = 0; c < CH_B; ++c) {
        const int ch = tid + c * NT;
        const int row = ch / (BK / VEC), kc = (ch % (BK / VEC)) * VEC;
        put16(Bs[buf][p], row * LDK + kc, rb[p][c]);
      }
    }
  };

  Acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc_zero<Tr>();

  const int lrow = lane & 15;
  const int lk = lane >> 4;

  if (nk > 0) {
    gload(kbeg);
    lstore(0);
    // the pipelined loop below keeps the register prefetch one slab ahead of
    // the LDS stores
    if constexpr (NS == 2 && NP == 1) gload(kbeg + min(1, nk - 1) * BK);
    __syncthreads();
  }
  if constexpr (NS == 2 && NP == 1) {
    // Software-pipelined slab loop (FP64 / FP32).  The operand fragments of
    // two MFMA steps are in registers or in flight at any time: after the
    // MFMAs of step s, the fragments of step s + 2 are read into the same
    // registers.  The last two steps of a slab read the first two of the next
    // slab, so the next slab's LDS stores go between the MFMA groups, and the
    // one barrier per slab sits before the last step, whose MFMAs then cover
    // the latency of the first reads from the new slab.  The global loads of
    // slab k + 2 are issued as soon as slab k + 1 is stored, so they have
    // about one slab of MFMAs to arrive.  The loop body has no branches (the
    // compiler's LDS wait counts are then those of the steady state): past
    // the last slab the prefetch reloads the last slab, and the stores and
    // reads go to the LDS buffer that is no longer read.
    constexpr int NKK = BK / Tr::KSTEP;
    static_assert(NKK >= 4 && NKK % 2 == 0, "pipelined loop needs an even step count >= 4");
    T fa[2][FM], fb[2][FN];
    auto fread = [&](int q, int b, int step) {
#pragma unroll
      for (int i = 0; i < FM; ++i) fa[q][i] = As[b][0][(wm0 + i * 16 + lrow) * LDK + step * Tr::KSTEP + lk];
#pragma unroll
      for (int j = 0; j < FN; ++j) fb[q][j] = Bs[b][0][(wn0 + j * 16 + lrow) * LDK + step * Tr::KSTEP + lk];
    };
    auto mma = [&](int q) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          if constexpr (sizeof(T) == 8)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[q][i], fb[q][j], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[q][i], fb[q][j], acc[i][j], 0, 0, 0);
        }
    };
    if (nk > 0) {
      // same order as in the loop (steps kept apart), so that the LDS wait
      // counts at the loop head stay those of the steady state
      fread(0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      fread(1, 0, 1);
      __builtin_amdgcn_sched_barrier(0);
    }
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
#pragma unroll
      for (int s = 0; s < NKK; ++s) {
        mma(s & 1);
        __builtin_amdgcn_sched_barrier(0);
        if (s + 2 < NKK) {
          fread(s & 1, cur, s + 2);
        } else {
          if (s == NKK - 2) __syncthreads();  // next slab stored; this one fully read
          fread(s & 1, cur ^ 1, s + 2 - NKK);
        }
        if (s == NKK - 3) {
          lstore(cur ^ 1);
          gload(kbeg + min(kt + 2, nk - 1) * BK);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  } else
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = NS == 2 ? (kt & 1) : 0;
    if (kt + 1 < nk) gload(kbeg + (kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += Tr::KSTEP) {
      if constexpr (NP == 1) {
        T a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = As[buf][0][(wm0 + i * 16 + lrow) * LDK + kk + lk];
#pragma unroll
        for (int j = 0; j < FN; ++j) b[j] = Bs[buf][0][(wn0 + j * 16 + lrow) * LDK + kk + lk];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if constexpr (sizeof(T) == 8)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
          }
      } else {
        bf8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          const int o = (wm0 + i * 16 + lrow) * LDK + kk + lk * 8;
          ah[i] = *reinterpret_cast<const bf8 *>(&As[buf][0][o]);
          al[i] = *reinterpret_cast<const bf8 *>(&As[buf][1][o]);
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int o = (wn0 + j * 16 + lrow) * LDK + kk + lk * 8;
          bh[j] = *reinterpret_cast<const bf8 *>(&Bs[buf][0][o]);
          bl[j] = *reinterpret_cast<const bf8 *>(&Bs[buf][1][o]);
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          }
      }
    }
    if (kt + 1 < nk) {
      if constexpr (NS == 1) __syncthreads();  // every wave is done with the slab
      lstore(NS == 2 ? buf ^ 1 : 0);
    }
    __syncthreads();
  }

  // --- epilogue: (m, n) -> permuted 4-index address ---------------------------
  const double alpha = P.alpha;
  double *C = P.C + (P.ksplit > 1 ? split * P.split_stride : 0);
  const int rdiv = P.rdiv;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn0 + j * 16 + lrow;
      if (n >= P.N) continue;
      const int64_t noff = (int64_t)(n / rdiv) * P.sn1 + (int64_t)(n % rdiv) * P.sn0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // accumulator item v of lane l is row (l/16) + 4v for the FP64 MFMA and
        // row 4(l/16) + v for the FP32 / BF16 ones; the column is l % 16
        const int m = m0 + wm0 + i * 16 + (sizeof(T) == 8 ? lk + 4 * v : lk * 4 + v);
        if (m >= P.M) continue;
        const int64_t off = (int64_t)(m / rdiv) * P.sm1 + (int64_t)(m % rdiv) * P.sm0 + noff;
        const double val = alpha * (double)acc[i][j][v];
        if (P.accumulate) C[off] += val; else C[off] = val;
      }
    }
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2:
// logical index of hardware workgroup hw in a grid of n, such that every XCD
// works through a contiguous range of logical indices.
__device__ inline int xcd_logical(int hw, int n) {
  const int xcd = hw % kNumXcd, kx = hw / kNumXcd;
  const int q8 = n / kNumXcd, rem8 = n % kNumXcd;
  return xcd < rem8 ? xcd * (q8 + 1) + kx : rem8 * (q8 + 1) + (xcd - rem8) * q8 + kx;
}

// Minimum waves per SIMD the register allocation must allow: the FP64 128 x 128
// tile (4 x 4 MFMA blocks per wave) is held to two so that two workgroups share
// a CU and hide each other's K-slab staging.
template <class Tr, int BM, int BN>
constexpr int gemm_wpe() { return (sizeof(typename Tr::T) == 8 && BM * BN >= 128 * 128) ? 2 : 1; }

// One workgroup per tile; the (at most kMaxGemmProbs) problems travel by value.
template <class Tr, int BM, int BN, int BK, int NS, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
gemm_nt_kernel(const GemmBatch batch) {
  const int bid = xcd_logical(blockIdx.x, batch.total_tiles);
  int lo = 0, hi = batch.nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (batch.seg_start[mid] <= bid) lo = mid; else hi = mid - 1;
  }
  gemm_tile<Tr, BM, BN, BK, NS>(batch.p[batch.seg_prob[lo]], batch.seg_local[lo] + bid - batch.seg_start[lo]);
}

// Persistent form for many problems: a grid sized to the resident capacity
// walks the global tile list (problems ordered by decreasing K, so the long
// tiles go first); workgroup w takes logical tiles w, w + G, w + 2G, ...
template <class Tr, int BM, int BN, int BK, int NS, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
gemm_nt_persistent(const GemmProb *__restrict__ probs, int count, int total) {
  const int G = gridDim.x;
  for (int t = xcd_logical(blockIdx.x, G); t < total; t += G) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (probs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const GemmProb P = probs[lo];
    gemm_tile<Tr, BM, BN, BK, NS>(P, t - P.tile_begin);
    __syncthreads();  // the next tile restages LDS
  }
}

// ---------------------------------------------------------------------------
// Configurations
// ---------------------------------------------------------------------------
namespace {
struct Cfg { int bm, bn, bk, ns; };
constexpr Cfg kCfgF64[] = {{128, 128, 16, 2}, {64, 64, 16, 2}, {128, 64, 16, 2}};
constexpr Cfg kCfgF32[] = {{128, 128, 32, 2}, {64, 64, 32, 2}, {128, 128, 64, 1}};
constexpr Cfg kCfgBF[] = {{128, 128, 32, 2}, {64, 64, 32, 2}, {128, 128, 64, 1}};

template <class Tr, int BM, int BN, int BK, int NS>
hipError_t launch_one(const GemmBatch &b, hipStream_t s) {
  hipLaunchKernelGGL((gemm_nt_kernel<Tr, BM, BN, BK, NS, gemm_wpe<Tr, BM, BN>()>), dim3(b.total_tiles),
                     dim3(256), 0, s, b);
  return hipGetLastError();
}

template <class Tr, int BM, int BN, int BK, int NS>
hipError_t launch_persistent(const GemmProb *dprobs, int count, int total, hipStream_t s) {
  static int grid = 0;  // resident workgroups on the whole device (per instantiation)
  if (grid == 0) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu,
          reinterpret_cast<const void *>(&gemm_nt_persistent<Tr, BM, BN, BK, NS, gemm_wpe<Tr, BM, BN>()>),
          256, 0);
    if (e != hipSuccess) return e;
    grid = std::max(kNumXcd, (cus * std::max(per_cu, 1)) / kNumXcd * kNumXcd);
  }
  const int g = std::min(grid, (int)round_up(total, kNumXcd));
  hipLaunchKernelGGL((gemm_nt_persistent<Tr, BM, BN, BK, NS, gemm_wpe<Tr, BM, BN>()>), dim3(g), dim3(256),
                     0, s, dprobs, count, total);
  return hipGetLastError();
}
}  // namespace

int gemm_num_tiles(GemmPrec) { return 3; }

GemmTileInfo gemm_tile_info(GemmPrec prec, int cfg) {
  const Cfg *t = prec == GEMM_F64 ? kCfgF64 : prec == GEMM_F32 ? kCfgF32 : kCfgBF;
  return {t[cfg].bm, t[cfg].bn, t[cfg].bk};
}

int gemm_default_cfg(GemmPrec prec, int M, int N) {
  // FP64 and split BF16: 128 x 128 tiles (the wide-K single-stage one for split
  // BF16) once a grouped launch of such products has a few per CU, 64 x 64
  // below.  FP32: the software-pipelined 64 x 64 tile at every size (at
  // r = 50 it beats both 128 x 128 shapes by about 10%).
  if (prec == GEMM_F32) return 1;
  const int64_t big = ((M + 127) / 128) * (int64_t)((N + 127) / 128);
  if (big < 128) return 1;
  return prec == GEMM_F64 ? 0 : 2;
}

hipError_t gemm_launch(GemmPrec prec, int cfg, GemmBatch &b, hipStream_t s) {
  const GemmTileInfo ti = gemm_tile_info(prec, cfg);
  int total = 0;
  for (int q = 0; q < b.count; ++q) {
    GemmProb &p = b.p[q];
    p.tiles_m = (p.M + ti.bm - 1) / ti.bm;
    p.tiles_n = (p.N + ti.bn - 1) / ti.bn;
    if (p.ksplit < 1) p.ksplit = 1;
    if (p.kchunk <= 0) p.kchunk = p.Kp;
    p.tile_begin = total;
    total += p.tiles_m * p.tiles_n * p.ksplit;
  }
  b.total_tiles = total;
  if (total == 0) return hipSuccess;
  b.nseg = 0;
  int start = 0;
  for (int c = 0; c < kGemmXcds; ++c)
    for (int q = 0; q < b.count; ++q) {
      const int n = b.p[q].tiles_m * b.p[q].tiles_n * b.p[q].ksplit;
      const int lo = (int)((int64_t)n * c / kGemmXcds), hi = (int)((int64_t)n * (c + 1) / kGemmXcds);
      if (hi <= lo) continue;
      b.seg_start[b.nseg] = start;
      b.seg_prob[b.nseg] = q;
      b.seg_local[b.nseg] = lo;
      ++b.nseg;
      start += hi - lo;
    }
  b.seg_start[b.nseg] = start;
#define ACSE_GEMM_CASE(TR, CFGS)                                                          \
  switch (cfg) {                                                                          \
    case 0: return launch_one<TR, CFGS[0].bm, CFGS[0].bn, CFGS[0].bk, CFGS[0].ns>(b, s);               \
    case 1: return launch_one<TR, CFGS[1].bm, CFGS[1].bn, CFGS[1].bk, CFGS[1].ns>(b, s);               \
    default: return launch_one<TR, CFGS[2].bm, CFGS[2].bn, CFGS[2].bk, CFGS[2].ns>(b, s);              \
  }
  if (prec == GEMM_F64) { ACSE_GEMM_CASE(TrF64, kCfgF64) }
  if (prec == GEMM_F32) { ACSE_GEMM_CASE(TrF32, kCfgF32) }
  ACSE_GEMM_CASE(TrBF16x3, kCfgBF)
#undef ACSE_GEMM_CASE
}

hipError_t gemm_launch_persistent(GemmPrec prec, int cfg, std::vector<GemmProb> &probs,
                                  GemmProb *host_stage, GemmProb *dprobs, hipStream_t s) {
  const GemmTileInfo ti = gemm_tile_info(prec, cfg);
  // longest K first; ties keep the caller's order
  std::stable_sort(probs.begin(), probs.end(),
                   [](const GemmProb &a, const GemmProb &b) { return a.Kp > b.Kp; });
  int total = 0;
  for (GemmProb &p : probs) {
    p.tiles_m = (p.M + ti.bm - 1) / ti.bm;
    p.tiles_n = (p.N + ti.bn - 1) / ti.bn;
    if (p.ksplit < 1) p.ksplit = 1;
    if (p.kchunk <= 0) p.kchunk = p.Kp;
    p.tile_begin = total;
    total += p.tiles_m * p.tiles_n * p.ksplit;
  }
  if (total == 0) return hipSuccess;
  const int count = (int)probs.size();
  std::copy(probs.begin(), probs.end(), host_stage);
  hipError_t e = hipMemcpyAsync(dprobs, host_stage, count * sizeof(GemmProb), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
#define ACSE_GEMM_CASE(TR, CFGS)                                                              \
  switch (cfg) {                                                                              \
    case 0: return launch_persistent<TR, CFGS[0].bm, CFGS[0].bn, CFGS[0].bk, CFGS[0].ns>(dprobs, count, total, s); \
    case 1: return launch_persistent<TR, CFGS[1].bm, CFGS[1].bn, CFGS[1].bk, CFGS[1].ns>(dprobs, count, total, s); \
    default: return launch_persistent<TR, CFGS[2].bm, CFGS[2].bn, CFGS[2].bk, CFGS[2].ns>(dprobs, count, total, s); \
  }
  if (prec == GEMM_F64) { ACSE_GEMM_CASE(TrF64, kCfgF64) }
  if (prec == GEMM_F32) { ACSE_GEMM_CASE(TrF32, kCfgF32) }
  ACSE_GEMM_CASE(TrBF16x3, kCfgBF)
#undef ACSE_GEMM_CASE
}

}  // namespace acse
