// Exact-accumulation products on the int8 MFMA (gemm_crt.hip): operand
// conversion to residue planes and the grouped modular product with its
// Chinese-remainder reconstruction.
#pragma once
#include "acse_internal.h"

namespace acse {

constexpr int kMinModuli = 8, kMaxModuli = 15, kDefaultModuli = 13;
constexpr int kCrtKPad = 256;  // residue rows are padded (with zeros) to a multiple of the K slab

// Moduli and reconstruction constants of a modulus count (host-built, passed by value).
struct CrtTable {
  int nmod;
  int m[kMaxModuli];      // moduli, pairwise coprime, <= 256
  int u[kMaxModuli];      // (M / m_j)^-1 mod m_j
  double log2M;
  double inv_m[kMaxModuli];
  double s1[kMaxModuli];  // M / m_j with its low bits cleared (<= 41 significant bits, exact)
  double s2[kMaxModuli];  // the rest of M / m_j (rounded)
  double M1, M2, inv_M;   // M = M1 + M2, M1 with <= 40 significant bits
};
bool crt_table(int nmod, CrtTable &T);
// Bits k of the scaled integers of a product over K terms: K 2^(2k) < M / 4.
int crt_kbits(const CrtTable &T, int K);
// Row stride (bytes) of a residue plane for K columns.
int64_t crt_ldr(int K);

// One FP64 operand [rows][ld] (K valid columns) -> exponents e[rows] and
// residue planes dst + j * plane, rows of ldr bytes.  premul: multiply by u_j.
struct ResidueJob {
  const double *src;
  int8_t *dst;
  int *e;
  int64_t plane;
  int row_begin;  // first block of this job in the launch
  int K, ld, ldr, kbits, premul;
};
constexpr int kMaxResidueJobs = 12;
struct ResidueBatch {
  ResidueJob job[kMaxResidueJobs];
  int count;
  int total_rows;
};
hipError_t launch_to_residues(const ResidueBatch &b, const CrtTable &T, hipStream_t s);

// Work of the modular product by XCD: entry e is every tile of problem
// prob[e] for modulus mod[e]; XCD c runs entries xs[c] .. xs[c+1]-1 in that
// order, entry e from its local tile start[e] on.
constexpr int kMaxModPairs = 6 * kMaxModuli;
struct ModSched {
  int xs[kGemmXcds + 1];
  int start[kMaxModPairs];
  uint8_t prob[kMaxModPairs], mod[kMaxModPairs];
};

// Grouped modular product: for each problem, A and B point at plane 0 of the
// residue operands (planes plane_a / plane_b bytes apart, rows of ld bytes,
// Kp = ld a multiple of kCrtKPad), and Y at crt_residue_out_bytes(M, N) bytes
// per modulus receives the residues of the product.  Fills in the batch's
// tile bookkeeping.
hipError_t gemm_crt_launch(GemmBatch &b, const CrtTable &T, hipStream_t s);
// Reconstruction of the batch launched by gemm_crt_launch (same stream, after
// it): from the residues in Y, ea / eb the row exponents and kshift = 2k,
// writes C through the store map.
hipError_t crt_combine_launch(const GemmBatch &b, const CrtTable &T, hipStream_t s);
int64_t crt_residue_out_bytes(int M, int N);

}  // namespace acse
