// Kernels of the residual map for states of any S_z (spin.hip): generic
// O(r^4) passes over spatial spin blocks (natural r^4 arrays [i][j][k][l]).
#pragma once
#include "acse_internal.h"
#include "tensor_ops.h"

namespace acse {

// One term of a linear combination: c * in[i s0 + j s1 + k s2 + l s3].
struct Term4 {
  const double *in;
  double c;
  int64_t s[4];
};
constexpr int kMaxTerms4 = 8;
struct Terms4 {
  Term4 t[kMaxTerms4];
  int n;
};
// Strides of a natural r^4 array read with its indices permuted: term index
// position d of the output reads source index position from[d].
inline Term4 term4(const double *in, double c, int r, int f0, int f1, int f2, int f3) {
  const int64_t nat[4] = {(int64_t)r * r * r, (int64_t)r * r, r, 1};
  return Term4{in, c, {nat[f0], nat[f1], nat[f2], nat[f3]}};
}

// out[i,j,k,l] (+)= sum_t c_t in_t[...]; with `mask` set, elements whose four
// spatial indices are all active are written as zero.
hipError_t launch_combine4(int r, const Terms4 &terms, double *out, int accumulate, const ActiveBits *mask,
                           hipStream_t s);
// GEMM operand [rows r^2][ld] with row (a,b), column (c,d) = sum_t c_t in_t[...]
// and the columns r^2 .. ld-1 zero.
hipError_t launch_pack_op4(int r, const Terms4 &terms, double *out, int ld, hipStream_t s);
// out[i,j,k,l] += c A[x_a0, x_a1] B[x_b0, x_b1], x = (i,j,k,l) and a0..b1
// positions in it (A, B r x r).
hipError_t launch_outer4(int r, double c, const double *A, int a0, int a1, const double *B, int b0, int b1,
                         double *out, hipStream_t s);
// out[k,s] (+)= sum_r in[k,r,r,s].
hipError_t launch_trace12(int r, const double *in, double *out, int accumulate, hipStream_t s);
// traces[q] = sum_{p,q'} in_q[p,q',p,q'] for q < count (count <= 8).
hipError_t launch_pair_traces(int r, int count, const double *const *in, double *traces, hipStream_t s);
// Step tail per spin block q < 3: d_q <- (d_q + eps U_q) tr0_q / (tr0_q + eps trU_q)
// with tr0 = traces[q], trU = traces[3 + q] (the trace of a sum is the sum of
// the traces).
hipError_t launch_spin_update(int r, double eps, double *const *d2, const double *const *U, const double *traces,
                              hipStream_t s);
// Natural r^4 array from a product whose rows ran over the pairs i < j of an
// antisymmetric pair (row-major, row stride ldc, columns (k,l) all r^2):
// out[i,j,k,l] = sign(i,j) C[pair(min,max)][k r + l], zero for i = j.
hipError_t launch_unpack_rows_lt(int r, const double *C, int64_t ldc, double *out, hipStream_t s);
// 1-RDM per spin from the new 2-RDM blocks: ga = c (Tr_2 d2aa + Tr_2 d2ab),
// gb = c (Tr_2 d2bb + Tr_1 d2ab), c = 2 / (N - 1).
hipError_t launch_spin_1rdm(int r, int N, const double *d2aa, const double *d2bb, const double *d2ab, double *ga,
                            double *gb, hipStream_t s);

// out = x + c y over n elements (out may be x).
hipError_t launch_spin_axpy(int64_t n, const double *x, double c, const double *y, double *out, hipStream_t s);

// ---- spin-orbital tensors of the NY share (n = 2r spin orbitals, alpha
// orbitals first: spin orbital p + r sigma) ------------------------------------
// Spin-block (bits b, bit 3 - t set when index t is beta) of a natural n^4
// array: out[(i + r s0), (j + r s1), (k + r s2), (l + r s3)] = c in[i,j,k,l].
hipError_t launch_so_embed(int r, int bits, const double *in, double c, double *out, hipStream_t s);
// The spin-orbital 2-cumulant of a state given by its spin blocks,
// c2[I,J,A,B] = 2D[I,J,A,B] - (1D[I,A] 1D[J,B] - 1D[J,A] 1D[I,B]) / 2 with 2D
// lifted from (d2aa, d2bb, d2ab) by the pair antisymmetry and 1D
// spin-diagonal (ga, gb), and cs = c2 with the third index scaled by sig[A].
hipError_t launch_so_cumulant(int r, const double *ga, const double *gb, const double *d2aa, const double *d2bb,
                              const double *d2ab, const double *sig, double *c2, double *cs, hipStream_t s);
// Y[k,a] = sum_p W[k,p,p,a] (n x n from a natural n^4 array).
hipError_t launch_so_trace_y(int n, const double *W, double *Y, hipStream_t s);
// B[i,j,k,l] += c sum_a Y[k,a] cs[i,j,a,l].
hipError_t launch_so_tpl(int n, double c, const double *Y, const double *cs, double *B, hipStream_t s);

// Spin-blocked GEMM operand from a natural n^4 array (n = 2r): operand
// position t reads the source with stride st[t]; the element with letter
// values (L0, L1, L2, L3) (spin s_t = L_t >= r, spatial l_t = L_t - s_t r) goes
// to row (2 s0 + s1) rpad + l0 r + l1, column (2 s2 + s3) kc + l2 r + l3 of a
// row-major buffer with ld = 4 kc.  Only the r^2 x r^2 part of each block is
// written (the padding is left as it is), and of it only the elements whose
// source element conserves spin: src_pos[t] is the source position operand
// position t reads, pair the source's conservation pair (spins of source
// positions {0, pair} against the other two); the other blocks are never read.
hipError_t launch_so_pack(int r, int64_t rpad, int64_t kc, const double *src, const int64_t st[4],
                          const int src_pos[4], int pair, double *out, hipStream_t s);

// ---- the NY share's adjoint on singlet states (spin-orbital, n = 2r) ---------
// X (all n^4 elements) from the fold's blocks: same-spin blocks Aaa, the
// (ab|ab) and (ba|ba) blocks Aab, the (ab|ba) and (ba|ab) blocks -Aab with the
// lower pair exchanged; zero elsewhere.
hipError_t launch_so_embed_singlet_x(int r, const double *Aaa, const double *Aab, double *X, hipStream_t s);
// Abaa += Xbar(aa|aa) + Xbar(bb|bb); Abab += Xbar(ab|ab) + Xbar(ba|ba)
// - Xbar(ab|ba) - Xbar(ba|ab) (the last two with the lower pair exchanged):
// the adjoint of the embedding above.
hipError_t launch_so_xbar_singlet(int r, const double *Xbar, double *Abaa, double *Abab, hipStream_t s);
// Adjoint of the singlet lift of the 2-RDM blocks, scaled by c and added:
// Gaa += c (D(aa|aa) + D(bb|bb)), Gab[p,q,s,t] += c (D(ab|ab)[p,q,s,t] +
// D(ba|ba)[q,p,t,s] - D(ab|ba)[p,q,t,s] - D(ba|ab)[q,p,s,t]).
hipError_t launch_so_dbar_singlet(int r, double c, const double *D, double *Gaa, double *Gab, hipStream_t s);
// Cotangent of B from that of F: Bbar = -Rbar + Rbar' + Rbar(k<->l) - Rbar'(k<->l)
// for sign = +1 (Hermitian X: F carries -C + C'), with the two exchanged terms
// negated for sign = -1; ' exchanges (ij) and (kl).  Rbar is nonzero on the
// (aa|aa) block (Rbar_aa) and the (ab|ab) block (Rbar_ab) only.
hipError_t launch_so_bbar(int r, const double *Rbar_aa, const double *Rbar_ab, double sign, double *Bbar,
                          hipStream_t s);
// Ybar[k,a] = c sum_{i,j,l} Bbar[i,j,k,l] cs[i,j,a,l] (fixed summation order).
// part: kSoYbarParts * n^2 / 2 doubles of scratch (the per-workgroup partial sums).
constexpr int kSoYbarParts = 512;
hipError_t launch_so_ybar(int n, double c, const double *Bbar, const double *cs, double *part, double *Ybar,
                          hipStream_t s);
// CSbar[i,j,a,l] += c sum_k Bbar[i,j,k,l] Y[k,a].
hipError_t launch_so_csbar_pl(int n, double c, const double *Bbar, const double *Y, double *CSbar, hipStream_t s);
// Wbar[k,p,p,a] += Ybar[k,a] for every p (adjoint of the trace Y = sum_p W[k,p,p,a]).
hipError_t launch_so_diag_add(int n, const double *Ybar, double *Wbar, hipStream_t s);
// C2bar += sig[a] CSbar, a the third index (adjoint of cs = sigma_a c2).
hipError_t launch_so_sigma_fold(int n, const double *sig, const double *CSbar, double *C2bar, hipStream_t s);
// gbar[x,y] += Dbar1[x,y] + Dbar1[x+r,y+r], the adjoint of the cumulant's
// wedge term through the 1-RDM diag(g, g):
// Dbar1[X,Y] = -1/2 [sum c[X,J,Y,Q] D1[J,Q] + sum c[I,X,R,Y] D1[I,R]
//                    - sum c[I,X,Y,Q] D1[I,Q] - sum c[X,J,R,Y] D1[J,R]].
hipError_t launch_so_d1bar_singlet(int r, const double *g, const double *C2bar, double *gbar, hipStream_t s);

}  // namespace acse
