// Launchers of the adjoint kernels (vjp.hip).
#pragma once
#include "tensor_ops.h"

namespace acse {

// dst[row][col] = c1 src1[...] + c2 src2[...], row = (a,b), col = (c,d) over r^2 x r^2,
// source index a*s[0] + b*s[1] + c*s[2] + d*s[3]; rows x ld output (zero padding
// unless accumulating).
struct PermArgs {
  int r;
  int64_t rows, ld;
  const double *src1;
  int64_t s1[4];
  double c1;
  const double *src2;  // may be null
  int64_t s2[4];
  double c2;
  int accumulate;      // FP64 output only: dst += value (padding untouched)
};
hipError_t launch_permute4(GemmPrec prec, const PermArgs &a, const OperandRef &out, hipStream_t s);
// Several permutes, each as launch_permute4 would run it, in as few launches
// as their destination types allow (up to kMaxPermJobs a launch).  The jobs
// must be independent: distinct destinations, and no job reads what another
// writes.
constexpr int kMaxPermJobs = 10;
hipError_t launch_permute4_batch(const GemmPrec *prec, const PermArgs *a, const OperandRef *out, int count,
                                 hipStream_t s);

// out[x,y] (+)= sum_t c_t sum_{u,v} T_t[x sx + y sy + u su + v sv] M_t[u*r + v]
struct ContractTerm {
  const double *T;
  int64_t sx, sy, su, sv;
  const double *M;
  double c;
};
constexpr int kMaxContractTerms = 6;
struct ContractArgs {
  ContractTerm term[kMaxContractTerms];
  int nterms;
};
// Terms with x, u in the first index pair of T and y, v in the second run as one
// pass over the slabs of T with partial vectors in `part` (2 r^3 doubles);
// other term patterns (or part == nullptr) take one block per output element.
struct SlabTerm {
  const double *T, *M;
  double c;
  int px, py;  // index positions of x (0 or 1) and y (2 or 3)
};
struct SlabContractArgs {
  SlabTerm term[kMaxContractTerms];
  int nterms;
};
hipError_t launch_contract42(int r, const ContractArgs &a, double *out, int accumulate, double *part,
                             hipStream_t s);

// Pair-packed operand of the pp adjoint products:
//   out[m][q] = sum_t c[t] src[t][a st[t][0] + b st[t][1] + c st[t][2] + d st[t][3]]
// row m = (a,b): any (a,b) with m = a r + b (rows_mode 0), a pair a < b
// (rows_mode 1) or a <= b (rows_mode 2) in packing order; column q = (c,d),
// c < d (k_le 0) or c <= d (k_le 1) in packing order; a term with offdiag[t]
// set is skipped where c = d.  Columns past the pair count up to ld are zero.
struct PairPackArgs {
  int r;
  int rows_mode;
  int k_le;
  int64_t ld;
  int nterms;  // 1..4
  const double *src[4];
  int64_t st[4][4];
  double c[4];
  int offdiag[4];
};
hipError_t launch_pack_pairs(GemmPrec prec, const PairPackArgs &a, const OperandRef &out, hipStream_t s);
// Natural r^4 tensor from a pair-packed product C (row stride ldc, columns lt
// pairs (r,s), antisymmetric in (r,s)): rows lt pairs (p,q), antisymmetric in
// (p,q) (rows_lt = 1), or all (p,q) (rows_lt = 0):
//   out[p,q,r,s] = sign(p,q) sign(r,s) C[row][col], zero where p = q (rows_lt) or r = s.
hipError_t launch_unpack_pairs(int r, int rows_lt, const double *C, int64_t ldc, double *out, hipStream_t s);
// Natural r^4 tensor from the two parts of a product split by the exchange
// r <-> s: Cp (columns le pairs, symmetric in (r,s)) and Cm (columns lt pairs,
// antisymmetric); rows all (p,q) (rows_packed 0), or le pairs of Cp and lt
// pairs of Cm with the same symmetry in (p,q) (rows_packed 1):
//   out[p,q,r,s] = (Cp[.][.] + sign(p,q) sign(r,s) Cm[.][.]) / 2, the Cm part zero where r = s or p = q.
hipError_t launch_unpack_pm(int r, int rows_packed, const double *Cp, int64_t ldp, const double *Cm, int64_t ldm,
                            double *out, hipStream_t s);

hipError_t launch_vjp_pe(int r, const double *Saa, const double *Sab, double *Ppb, double *Pmb,
                         double *E3b, hipStream_t s);
hipError_t launch_vjp_frank(int r, const double *fb, const double *g, double *Abaa, double *Abab,
                            hipStream_t s);
hipError_t launch_vjp_fold(int r, int N, const double *Abaa, const double *Abab, double *Vb_raw,
                           double *hb_raw, hipStream_t s);
enum ProjKind { PROJ_SYM2, PROJ_V, PROJ_AA, PROJ_AB };
hipError_t launch_proj(ProjKind k, int r, double c, const double *x, double *out, hipStream_t s);
hipError_t launch_identity(int r, double *I, hipStream_t s);

}  // namespace acse
