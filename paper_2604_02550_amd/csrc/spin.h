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

}  // namespace acse
