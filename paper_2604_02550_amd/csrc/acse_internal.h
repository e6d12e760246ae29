// Internal declarations shared by the HIP translation units of libacse.so.
#pragma once
#include <vector>
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstdint>

namespace acse {

// ---------------------------------------------------------------------------
// Grouped NT GEMM:  C_g[m, n] = alpha_g * sum_k A_g[m, k] * B_g[n, k]
//
// Operands are row-major with leading dimension ld (elements), rows padded to
// the tile height and K padded (with zeros) to a multiple of the K tile, so
// the kernel loads without bounds checks.  The store of element (m, n) goes to
//   C[(m / rdiv) * sm1 + (m % rdiv) * sm0 + (n / rdiv) * sn1 + (n % rdiv) * sn0]
// which lets the pair-index products write directly in any 4-index order.
// With ksplit > 1 each K chunk writes its own partial block at
// C + split * split_stride (natural layout m * N + n).
// ---------------------------------------------------------------------------
enum GemmPrec { GEMM_F64 = 0, GEMM_F32 = 1, GEMM_BF16X3 = 2, GEMM_I8CRT = 3 };

struct GemmProb {
  const void *A;      // plane 0 (hi for bf16x3)
  const void *B;
  const void *A2;     // lo plane (bf16x3 only)
  const void *B2;
  double *C;
  double alpha;
  int64_t sm1, sm0, sn1, sn0, split_stride;
  int M, N, Kp, ld;   // Kp: padded K (multiple of the K tile); ld >= Kp
  int rdiv;
  int ksplit, kchunk; // K chunks (kchunk multiple of the K tile)
  int tiles_m, tiles_n, tile_begin;
  int accumulate;     // 1: C += alpha * AB^T
  // exact-accumulation int8 products only (gemm_crt.hip): residue planes of A
  // and B lie plane_a / plane_b bytes apart, ea / eb are the row exponents
  // and kshift the total scaling bits 2k; u_out: neither operand carries the
  // reconstruction factors u_j, the product's residues are multiplied by them
  const int *ea;
  const int *eb;
  int64_t plane_a, plane_b;
  int kshift;
  int u_out;
  int8_t *Y;          // residues of the product per modulus: plane j at Y + j * plane_y,
  int64_t plane_y;    // rows grouped by four: byte (m / 4, n, m % 4)
};

constexpr int kMaxGemmProbs = 10;  // the by-value batch stays within the 4 KiB kernel-argument limit (2.3 KiB)
constexpr int kGemmXcds = 8;  // XCDs of the device, each with its own L2
// Logical tile order of a grouped launch: segment s (in order) covers logical
// tiles [seg_start[s], seg_start[s+1]) = tiles seg_local[s]... of problem
// seg_prob[s].  Segments take the c-th eighth of every problem for c = 0..7,
// so the contiguous logical range each XCD receives holds an equal share of
// every problem (balanced when the problems' K differ).
constexpr int kMaxGemmSegs = kMaxGemmProbs * kGemmXcds;
struct GemmBatch {
  GemmProb p[kMaxGemmProbs];
  int count;
  int total_tiles;
  int nseg;
  int seg_start[kMaxGemmSegs + 1];
  int seg_prob[kMaxGemmSegs];
  int seg_local[kMaxGemmSegs];
};

// Tile configurations (index = options.tile; -1 picks by size).
struct GemmTileInfo { int bm, bn, bk; };
int gemm_num_tiles(GemmPrec prec);
GemmTileInfo gemm_tile_info(GemmPrec prec, int cfg);
int gemm_default_cfg(GemmPrec prec, int M, int N);
// Row padding and K padding every operand buffer must provide.
constexpr int kRowPad = 256;
constexpr int kKPad = 64;

// Fills tiles_m/tiles_n/tile_begin/total_tiles and launches.
hipError_t gemm_launch(GemmPrec prec, int cfg, GemmBatch &batch, hipStream_t s);
// Persistent grouped launch over any number of problems: sorts `probs` in place
// by decreasing K, fills the tile counts, stages the descriptors through
// `host_stage` (pinned host memory the caller keeps until the copy has run)
// into `dprobs` (device) and launches one resident-size grid.
hipError_t gemm_launch_persistent(GemmPrec prec, int cfg, std::vector<GemmProb> &probs,
                                  GemmProb *host_stage, GemmProb *dprobs, hipStream_t s);

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace acse
