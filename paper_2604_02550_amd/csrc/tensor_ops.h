// Launchers of the O(r^4) / O(r^5) kernels (tensor_ops.hip).
#pragma once
#include "acse_internal.h"

namespace acse {

// A GEMM operand buffer: one plane (FP64/FP32) or a hi and a lo plane (BF16x3).
struct OperandRef {
  void *hi;
  void *lo;
};

// out[a, x, b] = alpha * sum_y M(x, y) (c1 in1 + c2 in2)[a, y, b]   (see tensor_ops.hip)
struct ModeArgs {
  int r;
  int64_t A, Bn;
  const double *in1;
  const double *in2;  // may be null
  double c1, c2;
  const double *g;    // r x r
  int transpose_m;    // M(x,y) = g[y][x] if set
  double alpha;
  int64_t adiv, so1, so0, sx, sb;
  int out_cols_fast;  // output contiguous along (a,b) columns rather than along x
  int accumulate;     // FP64 output only: out += result
  int wide;           // take the kernel shape of r > 64 (16-column panels, two
                      // row blocks per wave, K padded to 80 or 96) at any r
};
constexpr int kModeMaxR = 96;

hipError_t launch_fold(int r, int N, const double *h, const double *V, double *Aaa, double *Aab,
                       hipStream_t s);
hipError_t launch_w_natural(int r, const double *g, const double *d2aa, const double *d2ab,
                            double *Waa, double *Wab, hipStream_t s);
hipError_t launch_w_ph(GemmPrec prec, int r, int ld, const double *g, const double *d2aa,
                       const double *d2ab, const OperandRef &Rp, const OperandRef &Rm,
                       const OperandRef &R3, hipStream_t s);
// Packed pair indices over an r x r index square (row-major over the upper
// triangle):  lt: i < j,  p = i (2r - i - 1)/2 + (j - i - 1),  r(r-1)/2 pairs;
//             le: i <= j, p = i (2r - i + 1)/2 + (j - i),      r(r+1)/2 pairs.
__host__ __device__ inline int npair_lt(int r) { return r * (r - 1) / 2; }
__host__ __device__ inline int npair_le(int r) { return r * (r + 1) / 2; }
__host__ __device__ inline int pair_lt(int r, int i, int j) { return i * (2 * r - i - 1) / 2 + (j - i - 1); }
__host__ __device__ inline int pair_le(int r, int i, int j) { return i * (2 * r - i + 1) / 2 + (j - i); }
__device__ inline void unpair_le(int r, int p, int &i, int &j) {
  const double b = 2.0 * r + 1.0;
  int ii = (int)((b - sqrt(b * b - 8.0 * p)) * 0.5);
  if (ii < 0) ii = 0;
  while (ii > 0 && ii * (2 * r - ii + 1) / 2 > p) --ii;
  while ((ii + 1) * (2 * r - ii) / 2 <= p) ++ii;
  i = ii;
  j = ii + (p - ii * (2 * r - ii + 1) / 2);
}
// the lt pairs of r are the le pairs of r - 1 shifted by one column
__device__ inline void unpair_lt(int r, int p, int &i, int &j) {
  unpair_le(r - 1, p, i, j);
  ++j;
}
// leading dimensions (K padded to the GEMM K pad) of the packed pp operands
inline int64_t ld_pair_lt(int r) { return round_up(npair_lt(r), kKPad); }
inline int64_t ld_pair_le(int r) { return round_up(npair_le(r), kKPad); }

// Packed pp A operands D_aa, D_S, D_A (rows and K over pair indices).
hipError_t launch_d_operand(GemmPrec prec, int r, const double *d2aa, const double *d2ab,
                            const OperandRef &Daa, const OperandRef &DS, const OperandRef &DA,
                            hipStream_t s);
hipError_t launch_zero_kpad(GemmPrec prec, int r, int ld, const OperandRef &o, hipStream_t s);
hipError_t launch_f(int r, const double *Aaa, const double *Aab, const double *g, double *part,
                    double *f, hipStream_t s);
hipError_t launch_mode(GemmPrec prec, const ModeArgs &m, const OperandRef &out, hipStream_t s);
// ph A operands L+, L-, L3 (rows (k,i), K (p,s), leading dimension ld, K
// padding zeroed) in one pass over X_aa, X_ab, and optionally the partials
// [k][p][s] of f (as launch_f's first kernel); r <= kLopsMaxR (the register
// budget of two waves per SIMD; larger r use three one-index transforms).
constexpr int kLopsMaxR = 56;
hipError_t launch_lops(GemmPrec prec, int r, int ld, const double *g, const double *Xaa, const double *Xab,
                       const OperandRef &Lp, const OperandRef &Lm, const OperandRef &L3, double *fpart,
                       hipStream_t s);
// Largest violation of an input symmetry and largest magnitude -> out2[0], out2[1]
// (device); kind 0: symmetric r x r matrix, 1: (pq|rs) 8-fold, 2: alpha-alpha
// 2-RDM, 3: alpha-beta 2-RDM.  part: 2048 doubles of scratch (the Gram partials hold 512 r^2 >= 2048).
hipError_t launch_sym_check(int r, int kind, const double *x, double *part, double *out2, hipStream_t s);
// f[k,s] = sum_p part[k,p,s] (the second half of launch_f, for partials from launch_lops).
hipError_t launch_f_reduce(int r, const double *part, double *f, hipStream_t s);
// G2 (natural FP64) and the packed pp B operands B_aa, B_S, B_A.
hipError_t launch_g2(GemmPrec prec, int r, bool general, const double *Aaa, const double *Aab,
                     const double *Haa, const double *Hab, const double *f, double *G2aa, double *G2ab,
                     const OperandRef &Baa, const OperandRef &BS, const OperandRef &BA, hipStream_t s);
// G2 (never stored) fused with C^T[k,l,:,:] = alpha g G2[k,l,:,:] g for both
// blocks, and the packed pp B operands; r <= kG2cMaxR (the register budget
// of two waves per SIMD without spills).
constexpr int kG2cMaxR = 52;
hipError_t launch_g2c(GemmPrec prec, int r, const double *Aaa, const double *Aab, const double *Haa,
                      const double *Hab, const double *f, const double *g, double alpha, double *Caa, double *Cab,
                      const OperandRef &Baa, const OperandRef &BS, const OperandRef &BA, hipStream_t s);
// S from the packed pp products (Zaa [(i<j)][r^2], ZS [(i<=j)][r^2], ZA [(i<j)][r^2]),
// the particle-hole products and the gamma-t terms.
hipError_t launch_assemble(int r, bool general, const double *g, const double *t,
                           const double *Zaa, const double *ZS, const double *ZA, const double *Pp,
                           const double *Pm, const double *E3, double *Saa, double *Sab, hipStream_t s);
struct ActiveBits { uint64_t w[4]; };  // per-orbital active flags, r <= 256
hipError_t launch_finish(int r, double sigma, const double *Saa, const double *Sab,
                         const double *Caa, const double *Cab, double *Oaa, double *Oab,
                         const ActiveBits &active, double *Maa, double *Mab, double *partial,
                         double *sum_out, hipStream_t s);
int64_t finish_partials(int r);
hipError_t launch_t_reduce(int r, int nparts, const double *part, double *t, hipStream_t s,
                           int accumulate = 0);
// out[x,y] (+)= sum_z (w1 P1[x,z] Q1[y,z] + w2 P2[x,z] Q2[y,z]),  z in [0, r^3), P*,Q* natural [r][r^3].
// wide: use the kernel shape of the largest r (six 16-row blocks per side) at any r.
hipError_t launch_gram(int r, const double *P1, const double *Q1, double w1, const double *P2,
                       const double *Q2, double w2, double *part, double *out, int accumulate,
                       hipStream_t s, bool wide = false);
int t_partial_blocks();
// t[j,k] = sum_{prs} (W_aa[j,p,r,s] A_aa[k,p,r,s] + 2 W_ab[j,p,r,s] A_ab[k,p,r,s])
hipError_t launch_t(int r, const double *Waa, const double *Aaa, const double *Wab,
                    const double *Aab, double *part, double *t, hipStream_t s, bool wide = false);
hipError_t launch_energy(int r, int N, const double *h, const double *V, const double *d2aa,
                         const double *d2ab, double *partial, double *E_out, hipStream_t s);
// 2D <- (2D + eps U) rescaled to the input trace per block (in place), the
// traces [in_aa, in_ab, new_aa, new_ab] and the energy Tr(K 2D) of the result.
hipError_t launch_step_tail(int r, int N, double eps, const double *h, const double *V,
                            const double *Uaa, const double *Uab, double *d2aa, double *d2ab,
                            double *traces, double *partial, double *E_out, hipStream_t s);
hipError_t launch_traces(int r, const double *d2aa, const double *d2ab, double *traces,
                         hipStream_t s);
hipError_t launch_axpy2(int r, double eps, const double *aa, const double *ab, const double *Uaa,
                        const double *Uab, double *oaa, double *oab, hipStream_t s);
hipError_t launch_rescale(int r, const double *traces, const double *naa, const double *nab,
                          double *d2aa, double *d2ab, hipStream_t s);
hipError_t launch_contract_1rdm(int r, int N, const double *d2aa, const double *d2ab, double *g,
                                hipStream_t s);
hipError_t launch_fill(int64_t n, double v, double *p, hipStream_t s);
// oa = ca a, ob = cb b (n elements each).
hipError_t launch_scale2(int64_t n, double ca, const double *a, double cb, const double *b, double *oa,
                         double *ob, hipStream_t s);
// out[0] = sum_e a[e] b[e] in a fixed order (part: kDotBlocks doubles of scratch).
constexpr int kDotBlocks = 1024;
hipError_t launch_dot(int64_t n, const double *a, const double *b, double *part, double *out,
                      hipStream_t s);

}  // namespace acse
