// C ABI of libacse.so (declared in include/acse.h): context, validation and
// the orchestration of the residual map on the GPU.
//
// Residual map F(X) for a two-body tensor X with singlet blocks (A_aa, A_ab)
// (the antisymmetrised reduced Hamiltonian for the residual of Eq. (4), the
// masked residual for the update of Eq. (9)), with the Valdemoro 3-RDM of
// App. C, Eq. (C5) folded in and never formed:
//
//   f, t                 O(r^4), O(r^5) contractions of X with gamma and W
//   H, G2, Bpp = A - G2  one-index transforms and the f terms (pp operand)
//   Z_aa = Gamma2_aa Bpp_aa^T,  Z_ab = 2 Gamma2_ab Bpp_ab^T        pp GEMMs
//     (packed over the pair symmetries of Gamma2: Z_aa on pairs i<j with K over
//      r<s; Z_ab as its parts symmetric (i<=j, r<=s) and antisymmetric
//      (i<j, r<s) under the pair exchange)
//   P+- = (Xt_aa +- Xt_ab)(W'_a +- W'_b)^T,  E3 = -2 Xt3 W3^T      ph GEMMs
//   C = 4/3 (gamma x gamma) G2 (separable, two one-index transforms)
//   S = Z + C - gamma t terms - antisymmetrised particle-hole terms
//   F = S - S^T (Hermitian X),  F = S + S^T (anti-Hermitian X)
//
// The six products (about 7.5 r^6 flops) run as one grouped MFMA launch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <string>
#include <initializer_list>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/acse.h"
#include "gemm_crt.h"
#include "ny.h"
#include "ny_plan.h"
#include "spin.h"
#include "tensor_ops.h"
#include "vjp.h"

using namespace acse;

namespace {

constexpr int kNat = 26;     // natural r^4 arrays in Workspace
constexpr int kNumOps = 12;  // GEMM operand buffers in Workspace
constexpr int kProbsPerMap = 6;  // pair-index products of one residual map
constexpr int kTuneReps = 5;     // timed repetitions per tile configuration in the autotuners
constexpr int kAbPackMinR = 40;  // smallest r whose alpha-beta pp adjoint products run packed

// Residue planes and row exponents of the 12 operand buffers and the residues
// of the six products, for the int8 exact-accumulation products.
struct CrtWs {
  void *base = nullptr;
  int8_t *cres[12] = {};
  int *cexp[12] = {};
  int8_t *cy = nullptr;
};

struct Workspace {
  // natural FP64 r^4 arrays
  double *Aaa, *Aab, *Waa, *Wab, *Haa, *Hab, *G2aa, *G2ab, *T1, *Caa, *Cab;
  double *Zaa, *Zab, *Pp, *Pm, *E3, *Saa, *Sab;
  double *Raa, *Rab, *Maa, *Mab, *Uaa, *Uab, *Naa, *Nab;
  // GEMM operand buffers (sized for FP64, reused by the narrower formats)
  char *op[12];
  // small arrays
  double *fpart, *f, *tpart, *t, *partial, *scal;
  CrtWs *crt;  // residue buffers used with this workspace (int8 products)
};

}  // namespace

struct acse_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int r_max = 0;
  std::string err;
  void *base = nullptr;
  int64_t bytes = 0;
  int64_t op_bytes = 0;
  Workspace ws{};
  // stage timing
  bool profiling = false;
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double ms[ACSE_NUM_STAGES] = {};
  int64_t count[ACSE_NUM_STAGES] = {};
  std::map<std::pair<int, int>, int> tuned;  // (r, precision) -> tile configuration
  // ACSE_FLAG_GENERAL_KERNELS of the options of the call in progress (set by validate)
  bool general = false;
  // batched residual: one workspace per instance, sized for its own r
  void *bbase = nullptr;
  int64_t bbytes = 0;
  std::map<std::string, int> tuned_batch;  // "prec:r1,r2,..." -> tile configuration
  // side streams (default priority) for the per-instance stages of a batch
  hipStream_t side[4] = {};
  hipEvent_t fork_ev = nullptr, join_ev[4] = {};
  GemmProb *hdesc = nullptr;    // pinned staging of the persistent GEMM descriptors
  int hdesc_cap = 0;
  hipEvent_t hdesc_done = nullptr;  // recorded after the staging copy
  // adjoint workspace (allocated by the first VJP call)
  void *vbase = nullptr;
  int64_t vbytes = 0;
  double *vnat[36] = {};
  char *vop[12] = {};
  double *vsmall = nullptr;  // gb, tb, fb, I, hb_raw (r_max^2 each)
  // residues and row exponents of the adjoint's operand buffers and the
  // residues of one launch's products, for the int8 products (first such call)
  void *vcbase = nullptr;
  int8_t *vcres[12] = {};
  int *vcexp[12] = {};
  int8_t *vcy = nullptr;
  // Euler driver workspace (allocated by the first acse_solve call)
  void *sbase = nullptr;
  int64_t sbytes = 0;
  // Nakatsuji-Yasuda share (set by validate from the options of the call in
  // progress; workspace allocated by the first call that uses it, for r_max)
  bool ny_on = false;
  std::vector<double> ny_sigma;     // per spatial orbital, +1 / -1
  std::vector<double> ny_sigma_dev_copy;
  acse::ny::Plan ny_plan;
  bool ny_planned = false;
  void *nybase = nullptr;
  // residues of the NY operand buffers for the int8 products (first such call)
  void *nycbase = nullptr;
  std::vector<int8_t *> ny_cres;
  std::vector<int *> ny_cexp;
  int8_t *ny_cy = nullptr;
  int64_t nybytes = 0;
  int ny_r = 0;                     // r the operand buffers were last cleared for
  // set by acse_step around its update map: the 2-RDM has not changed since
  // the residual map, whose cumulant blocks and their operand layouts stand
  bool ny_reuse_d = false;
  // exact-accumulation int8 products (ACSE_INT8CRT): residue buffers of the
  // context's workspace and of the four batch lanes (each allocated by its
  // first use, for r_max and the largest modulus count) and the table of the
  // call's moduli
  CrtWs cw{};
  CrtWs lane_cw[4]{};
  CrtTable crt{};
  int crt_moduli = 0;      // modulus count of the call in progress (set by validate)
  // spin-block path for states of any S_z (allocated by its first call, for r_max)
  void *spbase = nullptr;
  int64_t spbytes = 0;
  void *spws = nullptr;    // its array table (a SpinWs)
  // spin-orbital tensors of the NY share of the spin-block path and of the NY
  // adjoint (an SoWs; allocated by the first such call for its r)
  void *sows = nullptr;
};

namespace {


acse_status fail(acse_ctx c, acse_status s, const std::string &msg) {
  if (c) c->err = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(ctx, ACSE_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

// Records one event pair around a stage when profiling is on.
struct StageTimer {
  acse_ctx c;
  int stage;
  hipEvent_t b = nullptr;
  StageTimer(acse_ctx c_, int stage_) : c(c_), stage(stage_) {
    if (!c->profiling) return;
    hipEvent_t a = take();
    b = take();
    if (a && b) {
      (void)hipEventRecord(a, c->stream);
      c->recs.push_back({stage, a, b});
    }
  }
  ~StageTimer() { stop(); }
  void stop() {
    if (c->profiling && b) (void)hipEventRecord(b, c->stream);
    b = nullptr;
  }
  hipEvent_t take() {
    if (!c->pool.empty()) { hipEvent_t e = c->pool.back(); c->pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int64_t op_rows(int r) { return round_up((int64_t)r * r, kRowPad); }
int64_t op_ld(int r) { return round_up((int64_t)r * r, kKPad); }

// Lays out the workspace for orbital count r from p (p == nullptr only sizes
// it); returns the bytes used.  `full` adds the step-only arrays (masked copy,
// update, new 2-RDM); without it they are null.
int64_t carve(char *p, int r, bool full, Workspace &w) {
  const int64_t r2 = (int64_t)r * r;
  const int64_t nat = round_up(r2 * r2 * 8, 256);
  const int64_t opb = round_up(op_rows(r) * op_ld(r) * 8, 256);
  char *q = p;
  auto take = [&](int64_t bytes) {
    char *x = q;
    q += bytes;
    return p ? x : nullptr;
  };
  double **nats[kNat] = {&w.Aaa, &w.Aab, &w.Waa, &w.Wab, &w.Haa, &w.Hab, &w.G2aa, &w.G2ab, &w.T1,
                         &w.Caa, &w.Cab, &w.Zaa, &w.Zab, &w.Pp,  &w.Pm,  &w.E3,  &w.Saa,  &w.Sab,
                         &w.Raa, &w.Rab, &w.Maa, &w.Mab, &w.Uaa, &w.Uab, &w.Naa, &w.Nab};
  const int nnat = full ? kNat : kNat - 6;
  for (int k = 0; k < kNat; ++k) *nats[k] = k < nnat ? reinterpret_cast<double *>(take(nat)) : nullptr;
  for (int k = 0; k < kNumOps; ++k) w.op[k] = take(opb);
  w.fpart = reinterpret_cast<double *>(take(round_up((int64_t)r * r2 * 8, 256)));
  w.f = reinterpret_cast<double *>(take(round_up(r2 * 8, 256)));
  w.tpart = reinterpret_cast<double *>(take(round_up((int64_t)t_partial_blocks() * r2 * 8, 256)));
  w.t = reinterpret_cast<double *>(take(round_up(r2 * 8, 256)));
  w.partial = reinterpret_cast<double *>(take(round_up(finish_partials(r) * 8, 256)));
  w.scal = reinterpret_cast<double *>(take(256));
  return q - p;
}

OperandRef operand(const Workspace &w, int idx, GemmPrec prec, int r) {
  OperandRef o{w.op[idx], nullptr};
  if (prec == GEMM_BF16X3) o.lo = w.op[idx] + op_rows(r) * op_ld(r) * 2;
  return o;
}
enum { OP_DAA, OP_DS, OP_DA, OP_BAA, OP_BS, OP_BA, OP_LP, OP_LM, OP_L3, OP_RP, OP_RM, OP_R3 };

// ACSE_FLAG_CHECK_INPUTS: the largest violation of each input's required
// symmetry, relative to the array's largest magnitude, must not exceed
// kSymTol (synchronises; partials in the Gram scratch, results in scal[16..]).
constexpr double kSymTol = 1e-12;

acse_status check_inputs(acse_ctx c, const acse_problem *p, bool need_d1) {
  HIP_TRY(c, hipSetDevice(c->device));
  struct Item { const double *x; int kind; const char *name, *what; };
  const Item items[5] = {
      {p->h, 0, "h", "symmetric"},
      {p->V, 1, "V", "invariant under p<->q, r<->s and (pq)<->(rs)"},
      {p->d2aa, 2, "d2aa", "antisymmetric under i<->j and k<->l and invariant under (ij)<->(kl)"},
      {p->d2ab, 3, "d2ab", "invariant under (ij)<->(kl) and (ij)(kl)->(ji)(lk)"},
      {p->d1, 0, "d1", "symmetric"}};
  const int n = need_d1 ? 5 : 4;
  Workspace &w = c->ws;
  for (int q = 0; q < n; ++q)
    HIP_TRY(c, launch_sym_check(p->r, items[q].kind, items[q].x, w.tpart, w.scal + 16 + 2 * q, c->stream));
  double host[10] = {};
  HIP_TRY(c, hipMemcpyAsync(host, w.scal + 16, 2 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int q = 0; q < n; ++q) {
    const double viol = host[2 * q], mag = host[2 * q + 1];
    if (!(viol <= kSymTol * mag)) {
      char buf[96];
      std::snprintf(buf, sizeof buf, ": largest violation %.3e against largest magnitude %.3e", viol, mag);
      return fail(c, ACSE_ERR_ARG, std::string(items[q].name) + " is not " + items[q].what + buf);
    }
  }
  return ACSE_OK;
}

acse_status validate(acse_ctx c, const acse_problem *p, const acse_options *o, bool need_d1 = true) {
  if (!c) return ACSE_ERR_ARG;
  if (!p) return fail(c, ACSE_ERR_ARG, "problem is NULL");
  if (p->r < 2 || p->r > c->r_max)
    return fail(c, ACSE_ERR_SHAPE, "r = " + std::to_string(p->r) + " outside [2, r_max = " +
                                       std::to_string(c->r_max) + "]");
  const int N = p->n_alpha + p->n_beta;
  if (p->n_alpha < 0 || p->n_beta < 0 || N < 2 || p->n_alpha > p->r || p->n_beta > p->r)
    return fail(c, ACSE_ERR_SHAPE, "electron counts must satisfy N >= 2 and n_sigma <= r");
  if (p->n_alpha != p->n_beta)
    return fail(c, ACSE_ERR_UNSUPPORTED, "n_alpha != n_beta: this call takes singlet blocks (use the _spin calls)");
  if (!p->h || !p->V || !p->d2aa || !p->d2ab || (need_d1 && !p->d1))
    return fail(c, ACSE_ERR_ARG, "a problem pointer is NULL");
  if (!aligned16(p->h) || !aligned16(p->V) || !aligned16(p->d2aa) || !aligned16(p->d2ab) ||
      (need_d1 && !aligned16(p->d1)))
    return fail(c, ACSE_ERR_ALIGN, "problem arrays must be 16-byte aligned");
  if (o) {
    if (o->precision < ACSE_FP64 || o->precision > ACSE_INT8CRT)
      return fail(c, ACSE_ERR_ARG, "unknown precision");
    if (o->moduli != 0 && (o->moduli < kMinModuli || o->moduli > kMaxModuli))
      return fail(c, ACSE_ERR_ARG, "moduli must be 0 or in [" + std::to_string(kMinModuli) + ", " +
                                       std::to_string(kMaxModuli) + "]");
    if (o->tile < -1 || o->tile >= gemm_num_tiles(GEMM_F64))
      return fail(c, ACSE_ERR_ARG, "tile configuration out of range");
    if (o->flags & ~(ACSE_FLAG_GENERAL_KERNELS | ACSE_FLAG_CHECK_INPUTS | ACSE_FLAG_BATCH_PERSISTENT))
      return fail(c, ACSE_ERR_ARG, "unknown option flags");
    if (o->reconstruction != ACSE_RECON_V && o->reconstruction != ACSE_RECON_NY)
      return fail(c, ACSE_ERR_ARG, "unknown reconstruction");
    if (o->reconstruction == ACSE_RECON_NY) {
      if (o->ny_sigma)
        for (int q = 0; q < p->r; ++q)
          if (o->ny_sigma[q] != 1 && o->ny_sigma[q] != -1)
            return fail(c, ACSE_ERR_ARG, "ny_sigma entries must be +1 or -1");
    }
  }
  c->general = o && (o->flags & ACSE_FLAG_GENERAL_KERNELS);
  c->crt_moduli = (o && o->precision == ACSE_INT8CRT) ? (o->moduli ? o->moduli : kDefaultModuli) : 0;
  c->ny_on = o && o->reconstruction == ACSE_RECON_NY;
  if (c->ny_on) {
    c->ny_sigma.assign(p->r, -1.0);
    for (int q = 0; q < p->r; ++q)
      c->ny_sigma[q] = o->ny_sigma ? (double)o->ny_sigma[q] : (q < p->n_alpha ? 1.0 : -1.0);
  }
  if (o && (o->flags & ACSE_FLAG_CHECK_INPUTS)) return check_inputs(c, p, need_d1);
  return ACSE_OK;
}

acse_status check_out(acse_ctx c, const void *p, const char *name) {
  if (!p) return fail(c, ACSE_ERR_ARG, std::string(name) + " is NULL");
  if (!aligned16(p)) return fail(c, ACSE_ERR_ALIGN, std::string(name) + " must be 16-byte aligned");
  return ACSE_OK;
}

GemmPrec prec_of(const acse_options *o) {
  if (!o) return GEMM_F64;
  switch (o->precision) {
    case ACSE_FP32: return GEMM_F32;
    case ACSE_BF16X3: return GEMM_BF16X3;
    case ACSE_INT8CRT: return GEMM_I8CRT;
    default: return GEMM_F64;
  }
}

// Format the operand producers write: the int8 exact-accumulation products take
// FP64 operands and convert them to residue planes afterwards.
GemmPrec op_prec(GemmPrec prec) { return prec == GEMM_I8CRT ? GEMM_F64 : prec; }

// Bytes of the six products' residues for one modulus at r (rows in fours).
int64_t crt_out_bytes_per_modulus(int r) {
  const int r2 = r * r;
  return 3 * crt_residue_out_bytes(r2, r2) + 2 * crt_residue_out_bytes(npair_lt(r), r2) +
         crt_residue_out_bytes(npair_le(r), r2);
}

// Allocates one residue workspace (first use), for r_max.
acse_status alloc_crt_ws(acse_ctx c, CrtWs &cw) {
  if (cw.base) return ACSE_OK;
  const int rm = c->r_max;
  const int64_t rows = op_rows(rm);
  const int64_t rbytes = round_up((int64_t)kMaxModuli * rows * crt_ldr(rm * rm), 256);
  const int64_t ebytes = round_up(rows * (int64_t)sizeof(int), 256);
  const int64_t ybytes = round_up(kMaxModuli * crt_out_bytes_per_modulus(rm), 256);
  const int64_t bytes = kNumOps * (rbytes + ebytes) + ybytes;
  if (hipMalloc(&cw.base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    cw.base = nullptr;
    return fail(c, ACSE_ERR_NOMEM, "cannot allocate the int8 residue workspace (" + std::to_string(bytes) + " bytes)");
  }
  char *q = static_cast<char *>(cw.base);
  for (int k = 0; k < kNumOps; ++k) {
    cw.cres[k] = reinterpret_cast<int8_t *>(q);
    q += rbytes;
    cw.cexp[k] = reinterpret_cast<int *>(q);
    q += ebytes;
  }
  cw.cy = reinterpret_cast<int8_t *>(q);
  return ACSE_OK;
}

// Residue workspace of the context's workspace (first use), and the moduli
// table of the call in progress.
acse_status ensure_crt(acse_ctx c) {
  acse_status st = alloc_crt_ws(c, c->cw);
  if (st != ACSE_OK) return st;
  c->ws.crt = &c->cw;
  if (c->crt.nmod != c->crt_moduli && !crt_table(c->crt_moduli, c->crt))
    return fail(c, ACSE_ERR_ARG, "no moduli table for " + std::to_string(c->crt_moduli) + " moduli");
  return ACSE_OK;
}

// Rows, K and leading dimension of operand buffer idx at r (the layouts of
// map_probs), and the K of the product it enters.
struct OpShape { int rows, K, ld; };
OpShape op_shape(int idx, int r) {
  const int r2 = r * r, nlt = npair_lt(r), nle = npair_le(r);
  const int ldlt = (int)ld_pair_lt(r), ldle = (int)ld_pair_le(r), ld = (int)op_ld(r);
  switch (idx) {
    case OP_DAA: return {nlt, nlt, ldlt};
    case OP_DS: return {nle, nle, ldle};
    case OP_DA: return {nlt, nlt, ldlt};
    case OP_BAA: return {r2, nlt, ldlt};
    case OP_BS: return {r2, nle, ldle};
    case OP_BA: return {r2, nlt, ldlt};
    default: return {r2, r2, ld};  // the ph operands L+-, L3, W'+-, W3
  }
}
int64_t crt_plane(int idx, int r) { return op_rows(r) * crt_ldr(op_shape(idx, r).K); }

// FP64 operands -> residue planes and row exponents.  rdm_side: the operands
// built from the 2-RDM (the ph B and pp A sides), which carry the
// reconstruction factors u_j; otherwise the X side (ph A and pp B).
acse_status crt_residues(acse_ctx c, const Workspace &w, int r, bool rdm_side) {
  static const int rdm_ops[6] = {OP_RP, OP_RM, OP_R3, OP_DAA, OP_DS, OP_DA};
  static const int x_ops[6] = {OP_LP, OP_LM, OP_L3, OP_BAA, OP_BS, OP_BA};
  const int *ops = rdm_side ? rdm_ops : x_ops;
  ResidueBatch b{};
  b.count = 6;
  int rows = 0;
  for (int q = 0; q < 6; ++q) {
    const int idx = ops[q];
    const OpShape sh = op_shape(idx, r);
    ResidueJob &J = b.job[q];
    J.src = reinterpret_cast<const double *>(w.op[idx]);
    J.dst = w.crt->cres[idx];
    J.e = w.crt->cexp[idx];
    J.plane = crt_plane(idx, r);
    J.row_begin = rows;
    J.K = sh.K;
    J.ld = sh.ld;
    J.ldr = (int)crt_ldr(sh.K);
    J.kbits = crt_kbits(c->crt, sh.K);
    J.premul = rdm_side ? 1 : 0;
    rows += sh.rows;
  }
  b.total_rows = rows;
  HIP_TRY(c, launch_to_residues(b, c->crt, c->stream));
  return ACSE_OK;
}

// Operands that depend only on (gamma, 2D): W natural, the ph B operands and
// the pp A operands.
acse_status prep_rdm_operands(acse_ctx c, const acse_problem *p, GemmPrec prec, Workspace &w);
acse_status prep_rdm_operands(acse_ctx c, const acse_problem *p, GemmPrec prec) {
  return prep_rdm_operands(c, p, prec, c->ws);
}
acse_status prep_rdm_operands(acse_ctx c, const acse_problem *p, GemmPrec prec, Workspace &w) {
  const int r = p->r;
  const int ld = (int)op_ld(r);
  StageTimer timer(c, 0);
  const GemmPrec op = op_prec(prec);
  HIP_TRY(c, launch_w_natural(r, p->d1, p->d2aa, p->d2ab, w.Waa, w.Wab, c->stream));
  HIP_TRY(c, launch_w_ph(op, r, ld, p->d1, p->d2aa, p->d2ab, operand(w, OP_RP, op, r),
                         operand(w, OP_RM, op, r), operand(w, OP_R3, op, r), c->stream));
  HIP_TRY(c, launch_d_operand(op, r, p->d2aa, p->d2ab, operand(w, OP_DAA, op, r),
                              operand(w, OP_DS, op, r), operand(w, OP_DA, op, r), c->stream));
  if (prec == GEMM_I8CRT) return crt_residues(c, w, r, true);
  return ACSE_OK;
}

ModeArgs mode_base(acse_ctx c, int r, const double *g) {
  ModeArgs m{};
  m.r = r;
  m.wide = c->general ? 1 : 0;
  m.g = g;
  m.c1 = 1.0;
  m.c2 = 0.0;
  m.alpha = 1.0;
  m.adiv = 1;
  return m;
}

// Stage 2 of F(X): the O(r^4)/O(r^5) transforms that feed the products.
acse_status map_front(acse_ctx c, const acse_problem *p, GemmPrec prec, const double *Xaa,
                      const double *Xab, Workspace &w) {
  if (prec == GEMM_I8CRT) {
    acse_status st = map_front(c, p, GEMM_F64, Xaa, Xab, w);
    if (st != ACSE_OK) return st;
    StageTimer t2(c, 2);
    return crt_residues(c, w, p->r, false);
  }
  const int r = p->r;
  const int64_t r2 = (int64_t)r * r, r3 = r2 * r;
  const int ld = (int)op_ld(r);
  const double *g = p->d1;
  hipStream_t s = c->stream;
  {
    StageTimer t2(c, 2);
    // ph A operands: L+-[(k,i),(p,s)] = sum_r g[i,r] (X_aa +- X_ab)[k,p,r,s],
    // L3[(k,j),(p,s)] = sum_r g[j,r] X_ab[k,p,s,r]; the one-pass kernel also
    // leaves the partials of f
    const bool lops = r <= kLopsMaxR && !c->general;
    if (lops) {
      HIP_TRY(c, launch_lops(prec, r, ld, g, Xaa, Xab, operand(w, OP_LP, prec, r), operand(w, OP_LM, prec, r),
                             operand(w, OP_L3, prec, r), w.fpart, s));
      HIP_TRY(c, launch_f_reduce(r, w.fpart, w.f, s));
    } else {
      HIP_TRY(c, launch_f(r, Xaa, Xab, g, w.fpart, w.f, s));
    }
    HIP_TRY(c, launch_t(r, w.Waa, Xaa, w.Wab, Xab, w.tpart, w.t, s, c->general));

    // H[k,l,(r,s)] = sum_p X[k,p,(r,s)] g[p,l]
    for (int b = 0; b < 2; ++b) {
      ModeArgs m = mode_base(c, r, g);
      m.A = r; m.Bn = r2; m.in1 = b ? Xab : Xaa; m.transpose_m = 1;
      m.so1 = r3; m.so0 = 0; m.sx = r2; m.sb = 1; m.out_cols_fast = 1;
      HIP_TRY(c, launch_mode(GEMM_F64, m, OperandRef{b ? w.Hab : w.Haa, nullptr}, s));
    }
    // G2, the packed pp B operands and C^T[k,l,i,j] = 4/3 sum_rs g_ir g_js G2[k,l,r,s]
    if (r <= kG2cMaxR && !c->general) {
      HIP_TRY(c, launch_g2c(prec, r, Xaa, Xab, w.Haa, w.Hab, w.f, g, 4.0 / 3.0, w.Caa, w.Cab,
                            operand(w, OP_BAA, prec, r), operand(w, OP_BS, prec, r),
                            operand(w, OP_BA, prec, r), s));
    } else {
      HIP_TRY(c, launch_g2(prec, r, c->general, Xaa, Xab, w.Haa, w.Hab, w.f, w.G2aa, w.G2ab,
                           operand(w, OP_BAA, prec, r), operand(w, OP_BS, prec, r),
                           operand(w, OP_BA, prec, r), s));
    }
    if (r > kG2cMaxR || c->general) for (int b = 0; b < 2; ++b) {
      ModeArgs m1 = mode_base(c, r, g);  // T1[k,l,r,j] = sum_s g[j,s] G2[k,l,r,s]
      m1.A = r3; m1.Bn = 1; m1.in1 = b ? w.G2ab : w.G2aa;
      m1.so1 = r; m1.so0 = 0; m1.sx = 1; m1.sb = 0; m1.out_cols_fast = 0;
      HIP_TRY(c, launch_mode(GEMM_F64, m1, OperandRef{w.T1, nullptr}, s));
      ModeArgs m2 = mode_base(c, r, g);  // C^T[k,l,i,j] = 4/3 sum_r g[i,r] T1[k,l,r,j]
      m2.A = r2; m2.Bn = r; m2.in1 = w.T1; m2.alpha = 4.0 / 3.0;
      m2.so1 = r2; m2.so0 = 0; m2.sx = r; m2.sb = 1; m2.out_cols_fast = 1;
      HIP_TRY(c, launch_mode(GEMM_F64, m2, OperandRef{b ? w.Cab : w.Caa, nullptr}, s));
    }
    if (lops) return ACSE_OK;
    // ph A operands by three one-index transforms
    for (int q : {OP_LP, OP_LM, OP_L3})
      HIP_TRY(c, launch_zero_kpad(prec, r, ld, operand(w, q, prec, r), s));
    for (int b = 0; b < 2; ++b) {
      ModeArgs m = mode_base(c, r, g);
      m.A = r2; m.Bn = r; m.in1 = Xaa; m.in2 = Xab; m.c2 = b ? -1.0 : 1.0;
      m.adiv = r; m.so1 = (int64_t)r * ld; m.so0 = r; m.sx = ld; m.sb = 1; m.out_cols_fast = 1;
      HIP_TRY(c, launch_mode(prec, m, operand(w, b ? OP_LM : OP_LP, prec, r), s));
    }
    {  // L3[(k,j),(p,s)] = sum_r g[j,r] X_ab[k,p,s,r]
      ModeArgs m = mode_base(c, r, g);
      m.A = r3; m.Bn = 1; m.in1 = Xab;
      m.adiv = r2; m.so1 = (int64_t)r * ld; m.so0 = 1; m.sx = ld; m.sb = 0; m.out_cols_fast = 1;
      HIP_TRY(c, launch_mode(prec, m, operand(w, OP_L3, prec, r), s));
    }
  }
  return ACSE_OK;
}

// K extent a product runs over: the operand buffers are zero from K to their
// row stride ld (a multiple of 64, the largest K tile of any precision), so a
// precision whose tile configurations all take smaller K tiles (FP64: 16)
// stops at the next multiple of its largest one instead of running over up to
// 63 columns of zeros.
int gemm_kp(GemmPrec prec, int K, int ld) {
  int bk = 1;
  for (int c = 0; c < gemm_num_tiles(prec); ++c) bk = std::max(bk, gemm_tile_info(prec, c).bk);
  return (int)std::min<int64_t>(ld, round_up(K, bk));
}

// The six pair-index products of F(X) as GEMM descriptors: three packed pp
// products (Z_aa over pairs i<j and K r<s; the alpha-beta block split into its
// parts symmetric (i<=j, r<=s) and antisymmetric (i<j, r<s) under the pair
// exchange) and the three ph products.
void map_probs(const Workspace &w, GemmPrec prec, int r, GemmProb *out) {
  const int64_t r2 = (int64_t)r * r, r3 = r2 * r;
  auto set = [&](int q, int ia, int ib, double alpha, double *C, int M, int K, int ld, int64_t sm1,
                 int64_t sm0, int64_t sn1, int64_t sn0) {
    GemmProb &P = out[q];
    P = GemmProb{};
    OperandRef a = operand(w, ia, prec, r), bb = operand(w, ib, prec, r);
    P.A = a.hi; P.A2 = a.lo; P.B = bb.hi; P.B2 = bb.lo;
    P.C = C; P.alpha = alpha;
    P.M = M; P.N = (int)r2; P.Kp = gemm_kp(prec, K, ld); P.ld = ld; P.rdiv = r;
    P.sm1 = sm1; P.sm0 = sm0; P.sn1 = sn1; P.sn0 = sn0;
    P.ksplit = 1; P.kchunk = P.Kp; P.accumulate = 0;
  };
  const int nlt = npair_lt(r), nle = npair_le(r);
  const int ldlt = (int)ld_pair_lt(r), ldle = (int)ld_pair_le(r), ld = (int)op_ld(r);
  // packed rows p -> C + p r^2 + (k r + l)
  set(0, OP_DAA, OP_BAA, 2.0, w.Zaa, nlt, nlt, ldlt, r3, r2, r, 1);
  set(1, OP_DS, OP_BS, 4.0, w.Zab, nle, nle, ldle, r3, r2, r, 1);
  set(2, OP_DA, OP_BA, 4.0, w.Zab + (int64_t)nle * r2, nlt, nlt, ldlt, r3, r2, r, 1);
  set(3, OP_LP, OP_RP, 1.0, w.Pp, (int)r2, (int)r2, ld, r, r3, r2, 1);    // rows (k,i), cols (j,l) -> [i,j,k,l]
  set(4, OP_LM, OP_RM, 1.0, w.Pm, (int)r2, (int)r2, ld, r, r3, r2, 1);
  set(5, OP_L3, OP_R3, -2.0, w.E3, (int)r2, (int)r2, ld, r, r2, r3, 1);   // rows (k,j), cols (i,l) -> [i,j,k,l]
}

// The same six products on the residue planes of the int8 exact-accumulation mode.
void map_probs_crt(acse_ctx c, const Workspace &w, int r, GemmProb *out) {
  map_probs(w, GEMM_F64, r, out);  // outputs, shapes, alphas and store maps
  static const int pa[6] = {OP_DAA, OP_DS, OP_DA, OP_LP, OP_LM, OP_L3};
  static const int pb[6] = {OP_BAA, OP_BS, OP_BA, OP_RP, OP_RM, OP_R3};
  int64_t yoff = 0;
  for (int q = 0; q < kProbsPerMap; ++q) {
    GemmProb &P = out[q];
    const int K = op_shape(pa[q], r).K;
    P.A = w.crt->cres[pa[q]];
    P.B = w.crt->cres[pb[q]];
    P.A2 = P.B2 = nullptr;
    P.ld = P.Kp = (int)crt_ldr(K);
    P.plane_a = crt_plane(pa[q], r);
    P.plane_b = crt_plane(pb[q], r);
    P.ea = w.crt->cexp[pa[q]];
    P.eb = w.crt->cexp[pb[q]];
    P.kshift = 2 * crt_kbits(c->crt, K);
    P.Y = w.crt->cy + yoff;
    P.plane_y = crt_residue_out_bytes(P.M, P.N);
    yoff += (int64_t)c->crt.nmod * P.plane_y;
  }
}

int map_cfg(acse_ctx c, GemmPrec prec, int r, int cfg) {
  if (cfg >= 0) return cfg;
  auto it = c->tuned.find({r, (int)prec});
  const int r2 = r * r;
  return it != c->tuned.end() ? it->second : gemm_default_cfg(prec, r2, r2);
}

// Nakatsuji-Yasuda workspace, sized for r_max: the seven source blocks and
// the nine product blocks (natural r^4), the operand buffers of the plan, an
// FP64 staging buffer per intermediate (FP32 / split-BF16 products write
// their first-stage results there, then one pass converts them to operand
// format), Y and sigma.  Operand buffers are cleared whenever r changes (their
// padding rows and columns must read as zero; the GEMMs and permutations
// write only the r^2 x r^2 part of the intermediates).
constexpr int kNySrc = 7, kNyProd = 12;  // 9 products + the 3 blocks of B
struct NyPtrs {
  double *src[kNySrc], *prod[kNyProd], *Y, *sig;
  std::vector<double *> buf;      // operand buffers
  std::vector<double *> staging;  // FP64 intermediates, in their next stage's operand layout
};

int64_t ny_num_bufs(const ny::Plan &P) { return (int64_t)P.num_bufs + (int64_t)P.staging.size(); }

NyPtrs ny_carve(acse_ctx c, int r) {
  NyPtrs q{};
  const int64_t rm = c->r_max;
  const int64_t nat = round_up(rm * rm * rm * rm * 8, 256);
  const int64_t opb = round_up(op_rows(r) * op_ld(r) * 8, 256);
  char *p = static_cast<char *>(c->nybase);
  for (int k = 0; k < kNySrc; ++k) { q.src[k] = reinterpret_cast<double *>(p); p += nat; }
  for (int k = 0; k < kNyProd; ++k) { q.prod[k] = reinterpret_cast<double *>(p); p += nat; }
  q.Y = reinterpret_cast<double *>(p); p += round_up(rm * rm * 8, 256);
  q.sig = reinterpret_cast<double *>(p); p += round_up(rm * 8, 256);
  q.buf.resize(c->ny_plan.num_bufs);
  for (int k = 0; k < c->ny_plan.num_bufs; ++k) { q.buf[k] = reinterpret_cast<double *>(p); p += opb; }
  q.staging.resize(c->ny_plan.staging.size());
  for (size_t k = 0; k < q.staging.size(); ++k) { q.staging[k] = reinterpret_cast<double *>(p); p += opb; }
  return q;
}

acse_status ensure_ny_ws(acse_ctx c) {
  if (!c->ny_planned) {
    c->ny_plan = ny::build_plan();
    c->ny_planned = true;
  }
  if (c->nybase) return ACSE_OK;
  const int64_t rm = c->r_max;
  const int64_t nat = round_up(rm * rm * rm * rm * 8, 256);
  const int64_t bytes = (kNySrc + kNyProd) * nat + round_up(rm * rm * 8, 256) + round_up(rm * 8, 256) +
                        ny_num_bufs(c->ny_plan) * c->op_bytes;
  if (hipMalloc(&c->nybase, bytes) != hipSuccess) {
    (void)hipGetLastError();
    c->nybase = nullptr;
    return fail(c, ACSE_ERR_NOMEM, "Nakatsuji-Yasuda workspace allocation failed");
  }
  c->nybytes = bytes;
  c->ny_r = 0;
  return ACSE_OK;
}

acse_status ny_share_run(acse_ctx c, const acse_problem *p, GemmPrec prec, int tile, const double *Xaa,
                         const double *Xab, double *Saa, double *Sab);

// Residue planes and row exponents of every NY operand buffer, and the
// residues of one launch's products, for the int8 products (first such call).
acse_status ensure_ny_crt(acse_ctx c) {
  if (!c->nycbase) {
    const int rm = c->r_max;
    const int nb = c->ny_plan.num_bufs;
    const int64_t r2 = (int64_t)rm * rm;
    const int64_t rbytes = round_up((int64_t)kMaxModuli * op_rows(rm) * crt_ldr((int)r2), 256);
    const int64_t ebytes = round_up(op_rows(rm) * (int64_t)sizeof(int), 256);
    const int64_t ybytes = round_up(6 * (int64_t)kMaxModuli * crt_residue_out_bytes((int)r2, (int)r2), 256);
    const int64_t bytes = nb * (rbytes + ebytes) + ybytes;
    if (hipMalloc(&c->nycbase, bytes) != hipSuccess) {
      (void)hipGetLastError();
      c->nycbase = nullptr;
      return fail(c, ACSE_ERR_NOMEM, "cannot allocate the int8 residue workspace of the NY share (" +
                                         std::to_string(bytes) + " bytes)");
    }
    char *q = static_cast<char *>(c->nycbase);
    c->ny_cres.assign(nb, nullptr);
    c->ny_cexp.assign(nb, nullptr);
    for (int k = 0; k < nb; ++k) {
      c->ny_cres[k] = reinterpret_cast<int8_t *>(q);
      q += rbytes;
      c->ny_cexp[k] = reinterpret_cast<int *>(q);
      q += ebytes;
    }
    c->ny_cy = reinterpret_cast<int8_t *>(q);
  }
  if (c->crt.nmod != c->crt_moduli && !crt_table(c->crt_moduli, c->crt))
    return fail(c, ACSE_ERR_ARG, "no moduli table for " + std::to_string(c->crt_moduli) + " moduli");
  return ACSE_OK;
}

// The NY share of F(X): S_aa -= C_aa, S_ab -= C_ab (C = B - B(k<->l), B the
// 3-cumulant's share of the 3-RDM contraction), on the plan of ny_plan.h.  No
// C++ exception (an allocation of the plan's containers, a plan lookup)
// leaves through the C interface.
acse_status ny_share(acse_ctx c, const acse_problem *p, GemmPrec prec, int tile, const double *Xaa,
                     const double *Xab, double *Saa, double *Sab) {
  try {
    return ny_share_run(c, p, prec, tile, Xaa, Xab, Saa, Sab);
  } catch (const std::exception &e) {
    return fail(c, ACSE_ERR_NOMEM, std::string("Nakatsuji-Yasuda share: ") + e.what());
  }
}

acse_status ny_share_run(acse_ctx c, const acse_problem *p, GemmPrec prec, int tile, const double *Xaa,
                         const double *Xab, double *Saa, double *Sab) {
  const int r = p->r;
  hipStream_t s = c->stream;
  StageTimer t6(c, 6);
  acse_status st = ensure_ny_ws(c);
  if (st != ACSE_OK) return st;
  // int8 exact accumulation: operands built in FP64, then converted to
  // residues; the products' residues carry the reconstruction factors (u_out)
  const bool crt = prec == GEMM_I8CRT;
  if (crt && (st = ensure_ny_crt(c)) != ACSE_OK) return st;
  if (crt) prec = GEMM_F64;
  const ny::Plan &P = c->ny_plan;
  NyPtrs q = ny_carve(c, r);
  const int64_t ld = op_ld(r), rows = op_rows(r), r2 = (int64_t)r * r;
  bool upload = c->ny_sigma_dev_copy != c->ny_sigma;
  if (c->ny_r != r) {
    const int64_t opb = round_up(rows * ld * 8, 256);
    HIP_TRY(c, launch_fill(ny_num_bufs(P) * opb / 8, 0.0, q.buf[0], s));
    c->ny_r = r;
    upload = true;
  }
  if (upload) {
    // the host vector lives in the context until the next change, after a synchronisation
    HIP_TRY(c, hipStreamSynchronize(s));
    c->ny_sigma_dev_copy = c->ny_sigma;
    HIP_TRY(c, hipMemcpyAsync(q.sig, c->ny_sigma_dev_copy.data(), r * sizeof(double), hipMemcpyHostToDevice, s));
  }
  // sources: X blocks 0000 / 0101 / 0110, then D and sigma D (kept from the
  // previous map of the same step when the 2-RDM has not changed)
  const bool keep_d = c->ny_reuse_d && !upload;
  HIP_TRY(c, launch_ny_sources(r, p->d1, p->d2aa, p->d2ab, Xab, q.sig, q.src, keep_d, s));
  const double *src[3][3] = {{Xaa, Xab, q.src[6]}, {q.src[0], q.src[1], q.src[2]}, {q.src[3], q.src[4], q.src[5]}};
  auto slot = [](int block) { return block == 0 ? 0 : block == 5 ? 1 : 2; };
  auto opref = [&](int id) {
    OperandRef o{q.buf[id], nullptr};
    if (prec == GEMM_BF16X3) o.lo = reinterpret_cast<char *>(q.buf[id]) + rows * ld * 2;
    return o;
  };
  auto stage_of = [&](int t, int b) { return q.staging[P.staging.at({t, b})]; };
  const int64_t nst[4] = {r2 * r, r2, r, 1};
  const int64_t pst[4] = {r * ld, ld, r, 1};  // staging: the operand layout in FP64
  int ns = 0;
  const ny::Stage *stg = ny::stages(&ns);
  const int cfg = map_cfg(c, prec, r, tile);
  const int kp = gemm_kp(prec, (int)r2, (int)ld);
  const int64_t ld_lt = ld_pair_lt(r);
  const int kp_lt = gemm_kp(prec, npair_lt(r), (int)ld_lt);
  for (int phase = 0; phase < 2; ++phase) {
    // operands of this phase: source blocks permuted into operand layout, or
    // intermediates converted from their FP64 staging; sums and differences
    // of two blocks for the crosswise pairs
    for (const ny::OperandBuild &o : P.operands) {
      if (o.phase != phase) continue;
      const bool src_op = ny::is_source(o.t1);
      if (keep_d && src_op && o.t1 != ny::T_X) continue;
      if (o.packed) {  // K over the pairs k0 < k1 of one source block
        if (!src_op || o.t2 >= 0) return fail(c, ACSE_ERR_UNSUPPORTED, "NY plan: unsupported packed operand");
        PairPackArgs pa{};
        pa.r = r;
        pa.rows_mode = 0;
        pa.k_le = 0;
        pa.ld = ld_lt;
        pa.nterms = 1;
        pa.src[0] = src[o.t1][slot(o.b1)];
        for (int t = 0; t < 4; ++t) pa.st[0][t] = nst[P.layout_strides[4 * o.layout + t]];
        pa.c[0] = 1.0;
        pa.offdiag[0] = 0;
        HIP_TRY(c, launch_pack_pairs(prec, pa, opref(o.buf), s));
        continue;
      }
      PermArgs a{};
      a.r = r;
      a.rows = rows;
      a.ld = ld;
      a.c1 = 1.0;
      if (src_op) {
        a.src1 = src[o.t1][slot(o.b1)];
        for (int t = 0; t < 4; ++t) a.s1[t] = nst[P.layout_strides[4 * o.layout + t]];
        if (o.t2 >= 0) {
          a.src2 = src[o.t2][slot(o.b2)];
          for (int t = 0; t < 4; ++t) a.s2[t] = a.s1[t];
          a.c2 = o.c2;
        }
      } else {
        a.src1 = stage_of(o.t1, o.b1);
        for (int t = 0; t < 4; ++t) a.s1[t] = pst[t];
        if (o.t2 >= 0) {
          a.src2 = stage_of(o.t2, o.b2);
          for (int t = 0; t < 4; ++t) a.s2[t] = pst[t];
          a.c2 = o.c2;
        }
      }
      HIP_TRY(c, launch_permute4(prec, a, opref(o.buf), s));
    }
    // int8 products: the residues of every operand buffer this phase reads
    // (K = r^2, or the r(r-1)/2 pairs of a packed operand); those of the
    // buffers built from D and sigma D alone are kept from the previous map
    // of the same step, like the buffers themselves (every buffer has its own
    // residue planes, and both maps run with the same moduli)
    std::vector<int> buf_packed(P.num_bufs, 0);
    std::vector<char> rdm_only(P.num_bufs, 0);
    for (const ny::OperandBuild &o : P.operands) {
      buf_packed[o.buf] = o.packed;
      rdm_only[o.buf] = ny::is_source(o.t1) && o.t1 != ny::T_X;
    }
    auto kdim = [&](int buf) { return buf_packed[buf] ? npair_lt(r) : (int)r2; };
    if (crt) {
      std::vector<char> used(P.num_bufs, 0);
      for (const ny::Product &g : P.products)
        if (g.phase == phase) used[g.a_buf] = used[g.b_buf] = 1;
      if (keep_d)
        for (int id = 0; id < P.num_bufs; ++id)
          if (rdm_only[id]) used[id] = 0;
      ResidueBatch rb{};
      int nrows = 0;
      for (int id = 0; id <= P.num_bufs; ++id) {
        if (id == P.num_bufs || rb.count == kMaxResidueJobs) {
          if (rb.count) {
            rb.total_rows = nrows;
            HIP_TRY(c, launch_to_residues(rb, c->crt, s));
          }
          rb = ResidueBatch{};
          nrows = 0;
          if (id == P.num_bufs) break;
        }
        if (!used[id]) continue;
        const int K = kdim(id);
        ResidueJob &J = rb.job[rb.count++];
        J.src = q.buf[id];
        J.dst = c->ny_cres[id];
        J.e = c->ny_cexp[id];
        J.plane = rows * crt_ldr(K);
        J.row_begin = nrows;
        J.K = K;
        J.ld = buf_packed[id] ? (int)ld_lt : (int)ld;
        J.ldr = (int)crt_ldr(K);
        J.kbits = crt_kbits(c->crt, K);
        J.premul = 0;
        nrows += (int)r2;
      }
    }
    // products: the t-th terms of all output blocks of the phase go out
    // together (distinct outputs), up to kMaxGemmProbs a launch (6 for the
    // int8 products; timed as their own stage)
    const size_t per_launch = crt ? 6 : kMaxGemmProbs;
    for (int term = 0;; ++term) {
      std::vector<const ny::Product *> round;
      for (const ny::Product &g : P.products)
        if (g.phase == phase && g.term == term) round.push_back(&g);
      if (round.empty()) break;
      for (size_t b0 = 0; b0 < round.size(); b0 += per_launch) {
        GemmBatch batch{};
        batch.count = (int)std::min<size_t>(per_launch, round.size() - b0);
        for (int k = 0; k < batch.count; ++k) {
          const ny::Product &g = *round[b0 + k];
          int64_t os[4];
          ny::gemm_out_strides(stg[g.stage], r, ld, os);
          GemmProb &G = batch.p[k];
          G = GemmProb{};
          const OperandRef ra = opref(g.a_buf), rb = opref(g.b_buf);
          G.A = ra.hi; G.A2 = ra.lo; G.B = rb.hi; G.B2 = rb.lo;
          G.C = ny::is_product(g.out) ? q.prod[P.product_nat.at({g.out, g.block})] : stage_of(g.out, g.block);
          G.alpha = g.alpha;
          G.M = (int)r2; G.N = (int)r2; G.rdiv = r;
          G.Kp = g.packed ? kp_lt : kp;
          G.ld = g.packed ? (int)ld_lt : (int)ld;
          G.sm1 = os[0]; G.sm0 = os[1]; G.sn1 = os[2]; G.sn0 = os[3];
          G.ksplit = 1; G.kchunk = G.Kp; G.accumulate = g.accumulate;
          if (crt) {
            const int K = kdim(g.a_buf);
            G.A = c->ny_cres[g.a_buf];
            G.B = c->ny_cres[g.b_buf];
            G.A2 = G.B2 = nullptr;
            G.ld = G.Kp = (int)crt_ldr(K);
            G.kchunk = G.Kp;
            G.plane_a = G.plane_b = rows * crt_ldr(K);
            G.ea = c->ny_cexp[g.a_buf];
            G.eb = c->ny_cexp[g.b_buf];
            G.kshift = 2 * crt_kbits(c->crt, K);
            G.u_out = 1;
            G.plane_y = crt_residue_out_bytes(G.M, G.N);
            G.Y = c->ny_cy + (int64_t)k * c->crt.nmod * G.plane_y;
          }
        }
        {
          StageTimer t7(c, 7);  // the block products alone (int8: the modular products)
          HIP_TRY(c, crt ? gemm_crt_launch(batch, c->crt, s) : gemm_launch(prec, cfg, batch, s));
        }
        if (crt) HIP_TRY(c, crt_combine_launch(batch, c->crt, s));
      }
    }
    for (const ny::Unscramble &u : P.unscrambles) {
      if (u.phase != phase) continue;
      if (ny::is_product(u.out)) {
        HIP_TRY(c, launch_ny_unscramble(r2 * r2, q.prod[P.product_nat.at({u.out, u.bx})],
                                        q.prod[P.product_nat.at({u.out, u.by})], s));
      } else {
        HIP_TRY(c, launch_ny_unscramble(r2 * ld, stage_of(u.out, u.bx), stage_of(u.out, u.by), s));
      }
    }
  }
  HIP_TRY(c, launch_ny_trace_y(r, ld, stage_of(ny::T_W, 0), stage_of(ny::T_W, 5), q.Y, s));
  NyCombineArgs a{};
  const int pblk[3] = {0, 5, 6};
  for (int b = 0; b < 3; ++b) {
    a.il[b] = q.prod[P.product_nat.at({ny::T_IL, pblk[b]})];
    a.ir[b] = q.prod[P.product_nat.at({ny::T_IR, pblk[b]})];
    a.pr[b] = q.prod[P.product_nat.at({ny::T_PR, pblk[b]})];
    a.sd[b] = q.src[3 + b];
  }
  a.Y = q.Y;
  for (int b = 0; b < 3; ++b) a.B[b] = q.prod[kNyProd - 3 + b];
  a.Saa = Saa;
  a.Sab = Sab;
  HIP_TRY(c, launch_ny_combine(r, a, s));
  return ACSE_OK;
}

// Stage 4 of F(X): assembly, (ij) <-> (kl) exchange, mask and the FP64 norm
// 2||O_aa||^2 + 4||O_ab||^2 into norm_out (device).  With the NY
// reconstruction its share joins the assembled sum before the exchange.
acse_status map_back(acse_ctx c, const acse_problem *p, double sigma, double *Oaa, double *Oab,
                     const ActiveBits &act, double *Maa, double *Mab, double *norm_out,
                     Workspace &w, const double *Xaa = nullptr, const double *Xab = nullptr,
                     GemmPrec prec = GEMM_F64, int tile = -1) {
  const int r = p->r;
  hipStream_t s = c->stream;
  {
    StageTimer t4(c, 4);
    HIP_TRY(c, launch_assemble(r, c->general, p->d1, w.t, w.Zaa, w.Zab,
                               w.Zab + (int64_t)npair_le(r) * r * r, w.Pp, w.Pm, w.E3, w.Saa, w.Sab, s));
  }
  if (c->ny_on) {
    if (!Xaa || !Xab) return fail(c, ACSE_ERR_UNSUPPORTED, "the NY share needs the map's X");
    acse_status st = ny_share(c, p, prec, tile, Xaa, Xab, w.Saa, w.Sab);
    if (st != ACSE_OK) return st;
  }
  StageTimer t4b(c, 4);
  HIP_TRY(c, launch_finish(r, sigma, w.Saa, w.Sab, w.Caa, w.Cab, Oaa, Oab, act, Maa, Mab,
                           w.partial, norm_out, s));
  return ACSE_OK;
}

// F(X) into (Oaa, Oab); sigma = -1 for Hermitian X, +1 for anti-Hermitian X.
// If Maa is not null it receives the active-masked copy.  The norm
// 2||O_aa||^2 + 4||O_ab||^2 lands in ws.scal[slot].
acse_status run_map(acse_ctx c, const acse_problem *p, GemmPrec prec, int cfg, const double *Xaa,
                    const double *Xab, double sigma, double *Oaa, double *Oab,
                    const ActiveBits &act, double *Maa, double *Mab, int slot) {
  const int r = p->r;
  const int64_t r2 = (int64_t)r * r;
  Workspace &w = c->ws;
  acse_status st = map_front(c, p, prec, Xaa, Xab, w);
  if (st != ACSE_OK) return st;
  GemmBatch batch{};
  batch.count = kProbsPerMap;
  if (prec == GEMM_I8CRT) {
    map_probs_crt(c, w, r, batch.p);
    {
      StageTimer t3(c, 3);
      HIP_TRY(c, gemm_crt_launch(batch, c->crt, c->stream));
    }
    {
      StageTimer t4(c, 4);  // the reconstruction writes the products' 4-index outputs
      HIP_TRY(c, crt_combine_launch(batch, c->crt, c->stream));
    }
    return map_back(c, p, sigma, Oaa, Oab, act, Maa, Mab, w.scal + slot, w, Xaa, Xab, prec, cfg);
  }
  map_probs(w, prec, r, batch.p);
  int use_cfg = cfg;
  if (use_cfg < 0) {
    auto it = c->tuned.find({r, (int)prec});
    use_cfg = it != c->tuned.end() ? it->second : gemm_default_cfg(prec, (int)r2, (int)r2);
  }
  {
    StageTimer t3(c, 3);
    HIP_TRY(c, gemm_launch(prec, use_cfg, batch, c->stream));
  }
  return map_back(c, p, sigma, Oaa, Oab, act, Maa, Mab, w.scal + slot, w, Xaa, Xab, prec, cfg);
}

ActiveBits make_bits(const acse_options *o, int r, bool *any) {
  ActiveBits b{};
  *any = false;
  if (o && o->active) {
    for (int q = 0; q < r; ++q)
      if (o->active[q]) { b.w[q >> 6] |= 1ull << (q & 63); *any = true; }
  }
  return b;
}

// The autotuners keep the size default unless another tile shape is at least
// kTuneMargin faster: the single-map timings they take are noisier than the
// differences between close configurations.
constexpr double kTuneMargin = 0.03;
int keep_default(int best_cfg, double best_ms, int default_cfg, const double *times_ms) {
  if (!times_ms || best_cfg == default_cfg) return best_cfg;
  return times_ms[default_cfg] <= best_ms * (1.0 + kTuneMargin) ? default_cfg : best_cfg;
}

const char *last_noctx_error();
void release_spin_ws(acse_ctx c);
void release_so_ws(acse_ctx c);

acse_status fetch_scalars(acse_ctx c, double *norm2_host, double *E_host) {
  if (!norm2_host && !E_host) return ACSE_OK;
  double host[2] = {0.0, 0.0};
  HIP_TRY(c, hipMemcpyAsync(host, c->ws.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (norm2_host) {
    *norm2_host = host[0];
    if (!std::isfinite(host[0])) return fail(c, ACSE_ERR_NONFINITE, "||R||^2 is not finite");
  }
  if (E_host) {
    *E_host = host[1];
    if (!std::isfinite(host[1])) return fail(c, ACSE_ERR_NONFINITE, "energy is not finite");
  }
  return ACSE_OK;
}

}  // namespace

extern "C" {

const char *acse_status_str(acse_status s) {
  switch (s) {
    case ACSE_OK: return "ACSE_OK";
    case ACSE_ERR_ARG: return "ACSE_ERR_ARG";
    case ACSE_ERR_SHAPE: return "ACSE_ERR_SHAPE";
    case ACSE_ERR_ALIGN: return "ACSE_ERR_ALIGN";
    case ACSE_ERR_UNSUPPORTED: return "ACSE_ERR_UNSUPPORTED";
    case ACSE_ERR_NOMEM: return "ACSE_ERR_NOMEM";
    case ACSE_ERR_HIP: return "ACSE_ERR_HIP";
    case ACSE_ERR_NONFINITE: return "ACSE_ERR_NONFINITE";
  }
  return "ACSE_ERR_UNKNOWN";
}

const char *acse_last_error(acse_ctx ctx) { return ctx ? ctx->err.c_str() : last_noctx_error(); }

int64_t acse_workspace_bytes(acse_ctx ctx) { return ctx ? ctx->bytes : -1; }

acse_status acse_create(acse_ctx *out, int device, void *hip_stream, int32_t r_max) {
  if (!out) return ACSE_ERR_ARG;
  *out = nullptr;
  if (r_max < 2 || r_max > kModeMaxR) return ACSE_ERR_SHAPE;
  acse_ctx c = new (std::nothrow) acse_ctx_s();
  if (!c) return ACSE_ERR_NOMEM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->r_max = r_max;
  if (hipSetDevice(device) != hipSuccess) { delete c; return ACSE_ERR_HIP; }
  Workspace &w = c->ws;
  c->bytes = carve(nullptr, r_max, true, w);
  c->op_bytes = round_up(op_rows(r_max) * op_ld(r_max) * 8, 256);
  if (hipMalloc(&c->base, c->bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return ACSE_ERR_NOMEM;
  }
  carve(static_cast<char *>(c->base), r_max, true, w);
  const int64_t opb = c->op_bytes;
  // Operand padding rows are read by full tiles: give every byte a defined value once.
  if (launch_fill((kNumOps * opb) / 8, 0.0, reinterpret_cast<double *>(w.op[0]), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipFree(c->base);
    delete c;
    return ACSE_ERR_HIP;
  }
  *out = c;
  return ACSE_OK;
}

acse_status acse_profile_enable(acse_ctx ctx, int32_t enable) {
  if (!ctx) return ACSE_ERR_ARG;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (auto &q : ctx->recs) { ctx->pool.push_back(q.a); ctx->pool.push_back(q.b); }
  ctx->recs.clear();
  for (int s = 0; s < ACSE_NUM_STAGES; ++s) { ctx->ms[s] = 0.0; ctx->count[s] = 0; }
  ctx->profiling = enable != 0;
  return ACSE_OK;
}

acse_status acse_profile_read(acse_ctx ctx, acse_profile_data *out) {
  if (!ctx || !out) return ACSE_ERR_ARG;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (auto &q : ctx->recs) {
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, q.a, q.b));
    ctx->ms[q.stage] += ms;
    ctx->count[q.stage] += 1;
    ctx->pool.push_back(q.a);
    ctx->pool.push_back(q.b);
  }
  ctx->recs.clear();
  for (int s = 0; s < ACSE_NUM_STAGES; ++s) { out->ms[s] = ctx->ms[s]; out->count[s] = ctx->count[s]; }
  return ACSE_OK;
}

acse_status acse_destroy(acse_ctx ctx) {
  if (!ctx) return ACSE_ERR_ARG;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto &q : ctx->recs) { (void)hipEventDestroy(q.a); (void)hipEventDestroy(q.b); }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->vbase) (void)hipFree(ctx->vbase);
  if (ctx->vcbase) (void)hipFree(ctx->vcbase);
  if (ctx->sbase) (void)hipFree(ctx->sbase);
  if (ctx->nybase) (void)hipFree(ctx->nybase);
  if (ctx->cw.base) (void)hipFree(ctx->cw.base);
  for (CrtWs &cw : ctx->lane_cw)
    if (cw.base) (void)hipFree(cw.base);
  if (ctx->spbase) (void)hipFree(ctx->spbase);
  if (ctx->nycbase) (void)hipFree(ctx->nycbase);
  release_spin_ws(ctx);
  release_so_ws(ctx);
  if (ctx->bbase) (void)hipFree(ctx->bbase);
  if (ctx->hdesc) (void)hipHostFree(ctx->hdesc);
  if (ctx->hdesc_done) (void)hipEventDestroy(ctx->hdesc_done);
  for (int q = 0; q < 4; ++q) {
    if (ctx->side[q]) (void)hipStreamDestroy(ctx->side[q]);
    if (ctx->join_ev[q]) (void)hipEventDestroy(ctx->join_ev[q]);
  }
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  (void)hipFree(ctx->base);
  delete ctx;
  return ACSE_OK;
}

acse_status acse_set_stream(acse_ctx ctx, void *hip_stream) {
  if (!ctx) return ACSE_ERR_ARG;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return ACSE_OK;
}

acse_status acse_residual(acse_ctx ctx, const acse_problem *prob, const acse_options *opts,
                          double *R_aa, double *R_ab, double *norm2_host) {
  acse_status st = validate(ctx, prob, opts);
  if (st != ACSE_OK) return st;
  if (ctx->crt_moduli && (st = ensure_crt(ctx)) != ACSE_OK) return st;
  if ((st = check_out(ctx, R_aa, "R_aa")) != ACSE_OK) return st;
  if ((st = check_out(ctx, R_ab, "R_ab")) != ACSE_OK) return st;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const GemmPrec prec = prec_of(opts);
  const int cfg = opts ? opts->tile : -1;
  if ((st = prep_rdm_operands(ctx, prob, prec)) != ACSE_OK) return st;
  const int N = prob->n_alpha + prob->n_beta;
  {
    StageTimer t1(ctx, 1);
    HIP_TRY(ctx, launch_fold(prob->r, N, prob->h, prob->V, ctx->ws.Aaa, ctx->ws.Aab, ctx->stream));
  }
  const ActiveBits none{};
  if ((st = run_map(ctx, prob, prec, cfg, ctx->ws.Aaa, ctx->ws.Aab, -1.0, R_aa, R_ab, none, nullptr,
                    nullptr, 0)) != ACSE_OK)
    return st;
  return fetch_scalars(ctx, norm2_host, nullptr);
}

acse_status acse_autotune(acse_ctx ctx, const acse_problem *prob, const acse_options *opts,
                          int32_t *best_tile, double *times_ms) {
  acse_status st = validate(ctx, prob, opts);
  if (st != ACSE_OK) return st;
  if (ctx->crt_moduli && (st = ensure_crt(ctx)) != ACSE_OK) return st;
  ctx->ny_on = false;  // the tile choice concerns the Valdemoro products; the NY ones share it
  if (!best_tile) return fail(ctx, ACSE_ERR_ARG, "best_tile is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const GemmPrec prec = prec_of(opts);
  const int r = prob->r;
  const int N = prob->n_alpha + prob->n_beta;
  Workspace &w = ctx->ws;
  if ((st = prep_rdm_operands(ctx, prob, prec)) != ACSE_OK) return st;
  HIP_TRY(ctx, launch_fold(r, N, prob->h, prob->V, w.Aaa, w.Aab, ctx->stream));
  // time the grouped GEMM of one residual map per configuration (profiling
  // state of the caller is saved and restored)
  const bool was = ctx->profiling;
  auto saved = std::move(ctx->recs);
  ctx->recs.clear();
  double best = 1e300;
  int arg = 0;
  double tms[ACSE_NUM_TILE_CONFIGS] = {};
  const ActiveBits none{};
  for (int cfg = 0; cfg < ACSE_NUM_TILE_CONFIGS; ++cfg) {
    ctx->profiling = false;
    if ((st = run_map(ctx, prob, prec, cfg, w.Aaa, w.Aab, -1.0, w.Raa, w.Rab, none, nullptr, nullptr,
                      0)) != ACSE_OK)
      break;
    ctx->profiling = true;
    for (int rep = 0; rep < kTuneReps; ++rep)
      if ((st = run_map(ctx, prob, prec, cfg, w.Aaa, w.Aab, -1.0, w.Raa, w.Rab, none, nullptr,
                        nullptr, 0)) != ACSE_OK)
        break;
    if (st != ACSE_OK) break;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) { st = fail(ctx, ACSE_ERR_HIP, "sync"); break; }
    double ms = 1e300;  // fastest of the timed repetitions (robust to interference)
    for (auto &q : ctx->recs) {
      if (q.stage == 3) {
        float e = 0.0f;
        (void)hipEventElapsedTime(&e, q.a, q.b);
        ms = std::min(ms, (double)e);
      }
      ctx->pool.push_back(q.a);
      ctx->pool.push_back(q.b);
    }
    ctx->recs.clear();
    tms[cfg] = ms;
    if (times_ms) times_ms[cfg] = ms;
    if (ms < best) { best = ms; arg = cfg; }
  }
  ctx->profiling = was;
  ctx->recs = std::move(saved);
  if (st != ACSE_OK) return st;
  arg = keep_default(arg, best, gemm_default_cfg(prec, r * r, r * r), tms);
  ctx->tuned[{r, (int)prec}] = arg;
  *best_tile = arg;
  return ACSE_OK;
}

acse_status acse_update_map(acse_ctx ctx, const acse_problem *prob, const acse_options *opts,
                            const double *X_aa, const double *X_ab, double *U_aa, double *U_ab) {
  acse_status st = validate(ctx, prob, opts);
  if (st != ACSE_OK) return st;
  if (ctx->crt_moduli && (st = ensure_crt(ctx)) != ACSE_OK) return st;
  if ((st = check_out(ctx, X_aa, "X_aa")) != ACSE_OK) return st;
  if ((st = check_out(ctx, X_ab, "X_ab")) != ACSE_OK) return st;
  if ((st = check_out(ctx, U_aa, "U_aa")) != ACSE_OK) return st;
  if ((st = check_out(ctx, U_ab, "U_ab")) != ACSE_OK) return st;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const GemmPrec prec = prec_of(opts);
  if ((st = prep_rdm_operands(ctx, prob, prec)) != ACSE_OK) return st;
  const ActiveBits none{};
  return run_map(ctx, prob, prec, opts ? opts->tile : -1, X_aa, X_ab, +1.0, U_aa, U_ab, none,
                 nullptr, nullptr, 2);
}

acse_status acse_energy(acse_ctx ctx, const acse_problem *prob, double *E_host) {
  acse_status st = validate(ctx, prob, nullptr, false);
  if (st != ACSE_OK) return st;
  if (!E_host) return fail(ctx, ACSE_ERR_ARG, "E_host is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const int N = prob->n_alpha + prob->n_beta;
  {
    StageTimer t5(ctx, 5);
    HIP_TRY(ctx, launch_energy(prob->r, N, prob->h, prob->V, prob->d2aa, prob->d2ab, ctx->ws.partial,
                               ctx->ws.scal + 1, ctx->stream));
  }
  return fetch_scalars(ctx, nullptr, E_host);
}

acse_status acse_step(acse_ctx ctx, acse_problem *prob, double eps, const acse_options *opts,
                      double *R_aa, double *R_ab, double *U_aa, double *U_ab, double *E_host,
                      double *norm2_host) {
  acse_status st = validate(ctx, prob, opts);
  if (st != ACSE_OK) return st;
  if (ctx->crt_moduli && (st = ensure_crt(ctx)) != ACSE_OK) return st;
  if (!std::isfinite(eps)) return fail(ctx, ACSE_ERR_ARG, "eps is not finite");
  for (const void *q : {static_cast<const void *>(R_aa), static_cast<const void *>(R_ab),
                        static_cast<const void *>(U_aa), static_cast<const void *>(U_ab)})
    if (q && !aligned16(q)) return fail(ctx, ACSE_ERR_ALIGN, "output arrays must be 16-byte aligned");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  Workspace &w = ctx->ws;
  hipStream_t s = ctx->stream;
  const int r = prob->r;
  const int N = prob->n_alpha + prob->n_beta;
  const GemmPrec prec = prec_of(opts);
  const int cfg = opts ? opts->tile : -1;
  double *Raa = R_aa ? R_aa : w.Raa, *Rab = R_ab ? R_ab : w.Rab;
  double *Uaa = U_aa ? U_aa : w.Uaa, *Uab = U_ab ? U_ab : w.Uab;
  bool masked = false;
  const ActiveBits act = make_bits(opts, r, &masked);

  if ((st = prep_rdm_operands(ctx, prob, prec)) != ACSE_OK) return st;
  {
    StageTimer t1(ctx, 1);
    HIP_TRY(ctx, launch_fold(r, N, prob->h, prob->V, w.Aaa, w.Aab, s));
  }
  // R = F(K), ||R||^2 -> scal[0], masked copy -> M
  if ((st = run_map(ctx, prob, prec, cfg, w.Aaa, w.Aab, -1.0, Raa, Rab, act,
                    masked ? w.Maa : nullptr, masked ? w.Mab : nullptr, 0)) != ACSE_OK)
    return st;
  // U = F(R_m), on the same 2-RDM
  ctx->ny_reuse_d = ctx->ny_on;
  st = run_map(ctx, prob, prec, cfg, masked ? w.Maa : Raa, masked ? w.Mab : Rab, +1.0, Uaa, Uab,
               ActiveBits{}, nullptr, nullptr, 2);
  ctx->ny_reuse_d = false;
  if (st != ACSE_OK) return st;
  // 2D <- 2D + eps U, trace restoration, 1-RDM contraction, energy (FP64)
  {
    StageTimer t5(ctx, 5);
    HIP_TRY(ctx, launch_step_tail(r, N, eps, prob->h, prob->V, Uaa, Uab, prob->d2aa, prob->d2ab,
                                  w.scal + 4, w.partial, w.scal + 1, s));
    HIP_TRY(ctx, launch_contract_1rdm(r, N, prob->d2aa, prob->d2ab, prob->d1, s));
  }
  return fetch_scalars(ctx, norm2_host, E_host);
}

}  // extern "C"

// ===========================================================================
// Residual without allocation.  The workspace of one residual map for r up to
// kNoAllocMaxR lives in a file-scope device array, so the call allocates no
// device memory: for callers that cannot call hipMalloc (stream capture into
// a HIP graph, allocation-free serving loops).
// ===========================================================================
namespace {
constexpr int kNoAllocMaxR = 16;
constexpr int64_t kNoAllocBytes = 24ll << 20;  // the residual workspace of r = 16 takes 17.9 MiB
constexpr int kNoAllocMaxDevices = 64;
}  // namespace

// One copy per GPU the library runs on, held until the process ends.  Host code
// never passes this name to a kernel (on the host it is a stand-in, not a
// device address); it uses the per-device address from hipGetSymbolAddress.
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {
thread_local std::string g_noctx_err;  // detail of the last failing context-free call

struct NoAllocSlot {
  std::once_flag once;
  char *ptr = nullptr;
  hipError_t err = hipSuccess;
};
NoAllocSlot g_noalloc[kNoAllocMaxDevices];

acse_status noalloc_fail(acse_status s, const std::string &msg) {
  g_noctx_err = msg;
  return s;
}
}  // namespace

namespace {
const char *last_noctx_error() { return g_noctx_err.c_str(); }
}  // namespace

extern "C" acse_status acse_residual_noalloc(void *hip_stream, const acse_problem *prob,
                                             const acse_options *opts, double *R_aa, double *R_ab,
                                             double *norm2_dev) {
  if (!prob) return noalloc_fail(ACSE_ERR_ARG, "problem is NULL");
  if (prob->r < 2 || prob->r > kNoAllocMaxR)
    return noalloc_fail(ACSE_ERR_SHAPE, "r = " + std::to_string(prob->r) +
                                            " outside [2, 16], the range of acse_residual_noalloc");
  if (opts && opts->reconstruction == ACSE_RECON_NY)
    return noalloc_fail(ACSE_ERR_UNSUPPORTED, "acse_residual_noalloc takes the Valdemoro reconstruction only");
  if (opts && opts->precision == ACSE_INT8CRT)
    return noalloc_fail(ACSE_ERR_UNSUPPORTED, "acse_residual_noalloc runs in FP64, FP32 or split BF16");
  if (norm2_dev && (reinterpret_cast<uintptr_t>(norm2_dev) & 7u))
    return noalloc_fail(ACSE_ERR_ALIGN, "norm2_dev must be 8-byte aligned");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return noalloc_fail(ACSE_ERR_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return noalloc_fail(ACSE_ERR_UNSUPPORTED, "device index " + std::to_string(dev) + " beyond 63");
  // the scratch address of this device, taken once with the device current
  NoAllocSlot &slot = g_noalloc[dev];
  std::call_once(slot.once, [&slot] {
    slot.err = hipGetSymbolAddress(reinterpret_cast<void **>(&slot.ptr), HIP_SYMBOL(scratch));
  });
  if (slot.err != hipSuccess || !slot.ptr)
    return noalloc_fail(ACSE_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(slot.err));
  // a context on the stack: the caller's stream, the workspace carved from the
  // scratch for this r, no profiling, no tuned tiles
  acse_ctx_s c;
  c.device = dev;
  c.stream = static_cast<hipStream_t>(hip_stream);
  c.r_max = kNoAllocMaxR;
  acse_status st = validate(&c, prob, opts);
  if (st == ACSE_OK) st = check_out(&c, R_aa, "R_aa");
  if (st == ACSE_OK) st = check_out(&c, R_ab, "R_ab");
  if (st != ACSE_OK) return noalloc_fail(st, c.err);
  const int r = prob->r;
  if (carve(nullptr, r, false, c.ws) > kNoAllocBytes)
    return noalloc_fail(ACSE_ERR_NOMEM, "the residual workspace exceeds the scratch array");
  carve(slot.ptr, r, false, c.ws);
  const GemmPrec prec = prec_of(opts);
  const int N = prob->n_alpha + prob->n_beta;
  if ((st = prep_rdm_operands(&c, prob, prec)) != ACSE_OK) return noalloc_fail(st, c.err);
  if (launch_fold(r, N, prob->h, prob->V, c.ws.Aaa, c.ws.Aab, c.stream) != hipSuccess)
    return noalloc_fail(ACSE_ERR_HIP, "fold launch failed");
  const ActiveBits none{};
  if ((st = run_map(&c, prob, prec, opts ? opts->tile : -1, c.ws.Aaa, c.ws.Aab, -1.0, R_aa, R_ab, none,
                    nullptr, nullptr, 0)) != ACSE_OK)
    return noalloc_fail(st, c.err);
  if (norm2_dev) {
    const hipError_t e = hipMemcpyAsync(norm2_dev, c.ws.scal, sizeof(double), hipMemcpyDeviceToDevice, c.stream);
    if (e != hipSuccess) return noalloc_fail(ACSE_ERR_HIP, std::string("norm copy: ") + hipGetErrorString(e));
  }
  return ACSE_OK;
}

// ===========================================================================
// Adjoint of the residual map (VJP).  The steps mirror the forward chain in
// reverse; every product of the forward has its two adjoint products here.
// ===========================================================================
namespace {

acse_status ensure_vjp_ws(acse_ctx c) {
  if (c->vbase) return ACSE_OK;
  const int64_t n4 = (int64_t)c->r_max * c->r_max * c->r_max * c->r_max;
  const int64_t r2 = (int64_t)c->r_max * c->r_max;
  const int64_t nat = round_up(n4 * 8, 256);
  const int64_t opb = c->op_bytes;
  const int64_t small = 5 * round_up(r2 * 8, 256);
  const int64_t bytes = 36 * nat + 12 * opb + small;
  if (hipMalloc(&c->vbase, bytes) != hipSuccess) {
    (void)hipGetLastError();
    c->vbase = nullptr;
    return fail(c, ACSE_ERR_NOMEM, "adjoint workspace allocation failed");
  }
  c->vbytes = bytes;
  char *p = static_cast<char *>(c->vbase);
  for (int q = 0; q < 36; ++q) { c->vnat[q] = reinterpret_cast<double *>(p); p += nat; }
  for (int q = 0; q < 12; ++q) { c->vop[q] = p; p += opb; }
  c->vsmall = reinterpret_cast<double *>(p);
  return ACSE_OK;
}

// Residue workspace of the adjoint's operand buffers (first int8 call) and
// the moduli table of the call in progress.
acse_status ensure_vjp_crt(acse_ctx c) {
  if (!c->vcbase) {
    const int rm = c->r_max;
    const int64_t r2 = (int64_t)rm * rm;
    const int64_t rbytes = round_up((int64_t)kMaxModuli * op_rows(rm) * crt_ldr((int)r2), 256);
    const int64_t ebytes = round_up(op_rows(rm) * (int64_t)sizeof(int), 256);
    const int64_t ybytes = round_up(6 * (int64_t)kMaxModuli * crt_residue_out_bytes((int)r2, (int)r2), 256);
    const int64_t bytes = 12 * (rbytes + ebytes) + ybytes;
    if (hipMalloc(&c->vcbase, bytes) != hipSuccess) {
      (void)hipGetLastError();
      c->vcbase = nullptr;
      return fail(c, ACSE_ERR_NOMEM, "cannot allocate the int8 residue workspace of the adjoint (" +
                                         std::to_string(bytes) + " bytes)");
    }
    char *q = static_cast<char *>(c->vcbase);
    for (int k = 0; k < 12; ++k) {
      c->vcres[k] = reinterpret_cast<int8_t *>(q);
      q += rbytes;
      c->vcexp[k] = reinterpret_cast<int *>(q);
      q += ebytes;
    }
    c->vcy = reinterpret_cast<int8_t *>(q);
  }
  if (c->crt.nmod != c->crt_moduli && !crt_table(c->crt_moduli, c->crt))
    return fail(c, ACSE_ERR_ARG, "no moduli table for " + std::to_string(c->crt_moduli) + " moduli");
  return ACSE_OK;
}

struct Nat4 {
  int64_t S[4];
  explicit Nat4(int r) {
    S[3] = 1; S[2] = r; S[1] = (int64_t)r * r; S[0] = (int64_t)r * r * r;
  }
  // strides of the source for destination index positions given by the source
  // positions they come from
  void map(const int m[4], int64_t out[4]) const {
    for (int d = 0; d < 4; ++d) out[d] = S[m[d]];
  }
};

// ---------------------------------------------------------------------------
// Spin-orbital tensors (n = 2r spin orbitals, alpha first) for the NY share of
// the spin-block map and for the NY adjoint: natural n^4 arrays, the two GEMM
// operands of one pairwise contraction, two n^2 and one n-sized arrays.
// Allocated by the first use for its n and array count, grown (after the
// stream has drained) when a later call needs more, kept until acse_destroy.
// ---------------------------------------------------------------------------
constexpr int kSoMaxR = 64;      // the operand relayout stages n = 2r rows of n + 1 doubles in LDS
constexpr int kSoMaxArrays = 12;
struct SoWs {
  void *base = nullptr;
  int n = 0, narr = 0;
  double *a[kSoMaxArrays] = {};
  double *opA = nullptr, *opB = nullptr, *Y = nullptr, *Yb = nullptr, *sig = nullptr;
  double *part = nullptr;        // kSoYbarParts * n^2 / 2 partial sums of Ybar
  std::vector<double> sig_host;  // what sig holds
  int op_r = 0;                  // r whose operand layout the padding of opA / opB was cleared for
  // int8 products (ACSE_INT8CRT): residue planes and row exponents of each of
  // the 16 (row spin pair, summed spin pair) sub-blocks of opA and opB, and
  // the residues of one launch's products; sized for c_r orbitals
  void *cbase = nullptr;
  int c_r = 0;
  int8_t *cres[2][16] = {};
  int *cexp[2][16] = {};
  int8_t *cy = nullptr;
};
constexpr int kSoCrtProbs = 6;  // products per modular launch

// Spin-blocked operand of r spatial orbitals: 4 row blocks of rpad rows, 4
// column chunks of kc columns (one per spin pair of the row / summed letters).
int64_t so_rpad(int r) { return round_up((int64_t)r * r, kRowPad); }
int64_t so_kc(int r) { return round_up((int64_t)r * r, kKPad); }
int64_t so_op_doubles(int r) { return 4 * so_rpad(r) * 4 * so_kc(r); }

acse_status ensure_so_ws(acse_ctx c, int n, int narr, SoWs *&out) {
  SoWs *w = static_cast<SoWs *>(c->sows);
  if (!w) {
    w = new (std::nothrow) SoWs();
    if (!w) return fail(c, ACSE_ERR_NOMEM, "cannot allocate the spin-orbital workspace table");
    c->sows = w;
  }
  out = w;
  if (w->base && w->n >= n && w->narr >= narr) return ACSE_OK;
  const int nn = std::max(n, w->n), na = std::max(narr, w->narr);
  if (w->base) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    (void)hipFree(w->base);
    w->base = nullptr;
    w->n = w->narr = 0;
  }
  const int64_t n2 = (int64_t)nn * nn;
  const int64_t nat = round_up(n2 * n2 * 8, 256), opb = round_up(so_op_doubles(nn / 2) * 8, 256);
  const int64_t sm = round_up(n2 * 8, 256);
  const int64_t pb = round_up((int64_t)kSoYbarParts * (n2 / 2) * 8, 256);
  const int64_t bytes = na * nat + 2 * opb + 2 * sm + round_up((int64_t)nn * 8, 256) + pb;
  if (hipMalloc(&w->base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    w->base = nullptr;
    return fail(c, ACSE_ERR_NOMEM, "cannot allocate the spin-orbital workspace of the NY share (" +
                                       std::to_string(bytes) + " bytes)");
  }
  char *q = static_cast<char *>(w->base);
  auto take = [&](int64_t b) { double *x = reinterpret_cast<double *>(q); q += b; return x; };
  for (int k = 0; k < na; ++k) w->a[k] = take(nat);
  w->opA = take(opb);
  w->opB = take(opb);
  w->Y = take(sm);
  w->Yb = take(sm);
  w->sig = take(round_up((int64_t)nn * 8, 256));
  w->part = take(pb);
  w->n = nn;
  w->narr = na;
  w->sig_host.clear();
  w->op_r = 0;
  return ACSE_OK;
}

// The residue workspace of the int8 spin-orbital products (first such call,
// or a larger r).
acse_status ensure_so_crt(acse_ctx c, SoWs &w, int r) {
  if (w.cbase && w.c_r >= r) return ACSE_OK;
  if (w.cbase) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    (void)hipFree(w.cbase);
    w.cbase = nullptr;
    w.c_r = 0;
  }
  const int64_t r2 = (int64_t)r * r, rpad = so_rpad(r);
  const int64_t rbytes = round_up((int64_t)kMaxModuli * rpad * crt_ldr((int)r2), 256);
  const int64_t ebytes = round_up(rpad * (int64_t)sizeof(int), 256);
  const int64_t ybytes = round_up(kSoCrtProbs * (int64_t)kMaxModuli * crt_residue_out_bytes((int)r2, (int)r2), 256);
  const int64_t bytes = 32 * (rbytes + ebytes) + ybytes;
  if (hipMalloc(&w.cbase, bytes) != hipSuccess) {
    (void)hipGetLastError();
    w.cbase = nullptr;
    return fail(c, ACSE_ERR_NOMEM, "cannot allocate the int8 residue workspace of the spin-orbital products (" +
                                       std::to_string(bytes) + " bytes)");
  }
  char *q = static_cast<char *>(w.cbase);
  for (int side = 0; side < 2; ++side)
    for (int k = 0; k < 16; ++k) {
      w.cres[side][k] = reinterpret_cast<int8_t *>(q);
      q += rbytes;
      w.cexp[side][k] = reinterpret_cast<int *>(q);
      q += ebytes;
    }
  w.cy = reinterpret_cast<int8_t *>(q);
  w.c_r = r;
  return ACSE_OK;
}

void release_so_ws(acse_ctx c) {
  SoWs *w = static_cast<SoWs *>(c->sows);
  if (w && w->cbase) (void)hipFree(w->cbase);
  if (w && w->base) (void)hipFree(w->base);
  delete w;
  c->sows = nullptr;
}

// The n spin-orbital occupations on the device (uploaded when they change;
// the host copy stays in the workspace until the next change, after a
// synchronisation).
acse_status so_upload_sigma(acse_ctx c, SoWs &w, const std::vector<double> &sig) {
  if (w.sig_host == sig) return ACSE_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  w.sig_host = sig;
  HIP_TRY(c, hipMemcpyAsync(w.sig, w.sig_host.data(), w.sig_host.size() * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  return ACSE_OK;
}

// Spin conservation of a spin-orbital tensor: an element is zero unless the
// beta count of positions {0, pair} equals that of the other two positions
// (pair = 1 for the tensors [upper pair][lower pair]; an intermediate such as
// sum_pr X^{kp}_{rq} cs^{jp}_{ar} -> [k,q,j,a] conserves over {0, 3}).
bool so_block_nonzero(int pair, const int sp[4]) {
  int o[2], k = 0;
  for (int t = 1; t < 4; ++t)
    if (t != pair) o[k++] = t;
  return sp[0] + sp[pair] == sp[o[0]] + sp[o[1]];
}

// out[lo] (+)= alpha sum A[la] B[lb] over natural n^4 arrays (n = 2r) whose
// axes carry the letters la, lb, lo (four distinct letters each): the two
// letters A and B share and lo lacks are summed.  pa, pb: the conservation
// pairs of A and B (so_block_nonzero).  Both operands are packed spin-block
// major ([spins of the two free letters][spins of the two summed letters],
// r^2 x r^2 blocks); one r^2 x r^2 x r^2 FP64 product runs per output spin
// block and summed spin pair whose A and B blocks both conserve spin, written
// through 4-index store strides into its spin block of out.  Without acc the
// output is cleared first (its blocks no product reaches stay zero).  crt:
// the products run on the int8 matrix cores in exact accumulation (the
// moduli of the call in progress): every operand sub-block a product reads
// is converted to residues with one exponent per row over its K = r^2
// columns, the products go out in launches of kSoCrtProbs, and each launch's
// reconstruction writes through the same store strides.
acse_status so_contract(acse_ctx c, SoWs &w, int n, double *out, const char *lo, const double *A, const char *la,
                        int pa, const double *B, const char *lb, int pb, double alpha, int acc = 0,
                        bool crt = false) {
  auto pos = [](const char *t, char ch) {
    for (int k = 0; k < 4; ++k)
      if (t[k] == ch) return k;
    return -1;
  };
  const int r = n / 2;
  const int64_t n2 = (int64_t)n * n, r2 = (int64_t)r * r;
  const int64_t pw[4] = {n2 * n, n2, n, 1};
  char fa[2], fb[2], kl[2];
  int nfa = 0, nfb = 0, nk = 0;
  for (int k = 0; k < 4; ++k) {
    const char ch = lo[k];
    const bool ia = pos(la, ch) >= 0, ib = pos(lb, ch) >= 0;
    if (ia == ib || (ia ? nfa : nfb) == 2) return fail(c, ACSE_ERR_HIP, "internal: bad spin-orbital contraction");
    (ia ? fa[nfa++] : fb[nfb++]) = ch;
  }
  for (int k = 0; k < 4; ++k) {
    const char ch = la[k];
    if (pos(lo, ch) >= 0) continue;
    if (pos(lb, ch) < 0 || nk == 2) return fail(c, ACSE_ERR_HIP, "internal: bad spin-orbital contraction");
    kl[nk++] = ch;
  }
  if (nfa != 2 || nfb != 2 || nk != 2) return fail(c, ACSE_ERR_HIP, "internal: bad spin-orbital contraction");
  hipStream_t s = c->stream;
  const int64_t rpad = so_rpad(r), kc = so_kc(r), ld = 4 * kc;
  if (w.op_r != r) {
    HIP_TRY(c, launch_fill(so_op_doubles(r), 0.0, w.opA, s));
    HIP_TRY(c, launch_fill(so_op_doubles(r), 0.0, w.opB, s));
    w.op_r = r;
  }
  auto pack = [&](const double *src, const char *ls, const char *f, int pair, double *dst) {
    const char order[4] = {f[0], f[1], kl[0], kl[1]};
    int64_t st[4];
    int sp[4];
    for (int k = 0; k < 4; ++k) {
      sp[k] = pos(ls, order[k]);
      st[k] = pw[sp[k]];
    }
    return launch_so_pack(r, rpad, kc, src, st, sp, pair, dst, s);
  };
  HIP_TRY(c, pack(A, la, fa, pa, w.opA));
  HIP_TRY(c, pack(B, lb, fb, pb, w.opB));
  if (!acc) HIP_TRY(c, launch_fill(n2 * n2, 0.0, out, s));
  // spin of each source position for a (free-pair, summed-pair) block
  auto nz = [&](const char *ls, const char *f, int pair, int RS, int KS) {
    int sp[4];
    sp[pos(ls, f[0])] = RS >> 1;
    sp[pos(ls, f[1])] = RS & 1;
    sp[pos(ls, kl[0])] = KS >> 1;
    sp[pos(ls, kl[1])] = KS & 1;
    return so_block_nonzero(pair, sp);
  };
  int ks[4][4][4], cnt[4][4] = {};
  for (int RS = 0; RS < 4; ++RS)
    for (int CS = 0; CS < 4; ++CS)
      for (int KS = 0; KS < 4; ++KS)
        if (nz(la, fa, pa, RS, KS) && nz(lb, fb, pb, CS, KS)) ks[RS][CS][cnt[RS][CS]++] = KS;
  const int cfg = gemm_default_cfg(GEMM_F64, (int)r2, (int)r2);
  const int kp = gemm_kp(GEMM_F64, (int)r2, (int)kc);
  const int64_t sm1 = pw[pos(lo, fa[0])], sm0 = pw[pos(lo, fa[1])];
  const int64_t sn1 = pw[pos(lo, fb[0])], sn0 = pw[pos(lo, fb[1])];
  if (crt) {
    acse_status st = ensure_so_crt(c, w, r);
    if (st != ACSE_OK) return st;
    const int K = (int)r2;
    const int64_t ldr = crt_ldr(K), plane = rpad * ldr, plane_y = crt_residue_out_bytes(K, K);
    const int kbits = crt_kbits(c->crt, K);
    bool need[2][16] = {};
    for (int RS = 0; RS < 4; ++RS)
      for (int CS = 0; CS < 4; ++CS)
        for (int t = 0; t < cnt[RS][CS]; ++t) {
          need[0][RS * 4 + ks[RS][CS][t]] = true;
          need[1][CS * 4 + ks[RS][CS][t]] = true;
        }
    ResidueBatch rb{};
    int nrows = 0;
    for (int side = 0; side < 2; ++side)
      for (int q = 0; q < 16; ++q) {
        if (!need[side][q]) continue;
        if (rb.count == kMaxResidueJobs) {
          rb.total_rows = nrows;
          HIP_TRY(c, launch_to_residues(rb, c->crt, s));
          rb = ResidueBatch{};
          nrows = 0;
        }
        ResidueJob &J = rb.job[rb.count++];
        J.src = (side ? w.opB : w.opA) + (q >> 2) * rpad * ld + (q & 3) * kc;
        J.dst = w.cres[side][q];
        J.e = w.cexp[side][q];
        J.plane = plane;
        J.row_begin = nrows;
        J.K = K;
        J.ld = (int)ld;
        J.ldr = (int)ldr;
        J.kbits = kbits;
        J.premul = 0;
        nrows += K;
      }
    if (rb.count) {
      rb.total_rows = nrows;
      HIP_TRY(c, launch_to_residues(rb, c->crt, s));
    }
    // round t: the t-th summed spin pair of every output block; a launch never
    // spans two rounds, so that no launch holds two products of one output
    for (int t = 0; t < 4; ++t) {
      GemmBatch b{};
      b.count = 0;
      for (int RS = 0; RS < 4; ++RS)
        for (int CS = 0; CS < 4; ++CS) {
          if (cnt[RS][CS] <= t) continue;
          const int KS = ks[RS][CS][t];
          GemmProb &P = b.p[b.count];
          P = GemmProb{};
          P.A = w.cres[0][RS * 4 + KS];
          P.B = w.cres[1][CS * 4 + KS];
          P.C = out + (RS >> 1) * r * sm1 + (RS & 1) * r * sm0 + (CS >> 1) * r * sn1 + (CS & 1) * r * sn0;
          P.alpha = alpha;
          P.M = K; P.N = K; P.ld = P.Kp = (int)ldr; P.rdiv = r;
          P.sm1 = sm1; P.sm0 = sm0; P.sn1 = sn1; P.sn0 = sn0;
          P.ksplit = 1; P.kchunk = P.Kp; P.accumulate = (t == 0 && !acc) ? 0 : 1;
          P.plane_a = P.plane_b = plane;
          P.ea = w.cexp[0][RS * 4 + KS];
          P.eb = w.cexp[1][CS * 4 + KS];
          P.kshift = 2 * kbits;
          P.u_out = 1;
          P.plane_y = plane_y;
          P.Y = w.cy + (int64_t)b.count * c->crt.nmod * plane_y;
          if (++b.count == kSoCrtProbs) {
            {
              StageTimer t7(c, 7);  // the modular products alone
              HIP_TRY(c, gemm_crt_launch(b, c->crt, s));
            }
            HIP_TRY(c, crt_combine_launch(b, c->crt, s));
            b = GemmBatch{};
            b.count = 0;
          }
        }
      if (b.count) {
        {
          StageTimer t7(c, 7);
          HIP_TRY(c, gemm_crt_launch(b, c->crt, s));
        }
        HIP_TRY(c, crt_combine_launch(b, c->crt, s));
      }
    }
    return ACSE_OK;
  }
  StageTimer t7(c, 7);  // the products alone
  // round t: the t-th summed spin pair of every output block (distinct outputs per launch)
  for (int t = 0; t < 4; ++t) {
    GemmBatch b{};
    b.count = 0;
    for (int RS = 0; RS < 4; ++RS)
      for (int CS = 0; CS < 4; ++CS) {
        if (cnt[RS][CS] <= t) continue;
        const int KS = ks[RS][CS][t];
        GemmProb &P = b.p[b.count++];
        P = GemmProb{};
        P.A = w.opA + RS * rpad * ld + KS * kc;
        P.B = w.opB + CS * rpad * ld + KS * kc;
        P.C = out + (RS >> 1) * r * sm1 + (RS & 1) * r * sm0 + (CS >> 1) * r * sn1 + (CS & 1) * r * sn0;
        P.alpha = alpha;
        P.M = (int)r2; P.N = (int)r2; P.ld = (int)ld; P.Kp = kp; P.rdiv = r;
        P.sm1 = sm1; P.sm0 = sm0; P.sn1 = sn1; P.sn0 = sn0;
        P.ksplit = 1; P.kchunk = kp; P.accumulate = (t == 0 && !acc) ? 0 : 1;
        if (b.count == kMaxGemmProbs) {
          HIP_TRY(c, gemm_launch(GEMM_F64, cfg, b, s));
          b = GemmBatch{};
          b.count = 0;
        }
      }
    if (b.count) HIP_TRY(c, gemm_launch(GEMM_F64, cfg, b, s));
  }
  return ACSE_OK;
}

Term4 so_term(const double *in, double cf, int64_t s0, int64_t s1, int64_t s2, int64_t s3) {
  Term4 t{};
  t.in = in; t.c = cf; t.s[0] = s0; t.s[1] = s1; t.s[2] = s2; t.s[3] = s3;
  return t;
}

// The NY share's adjoint on the singlet residual (R = S - S^T, X = the fold's
// X_A embedded as a spin-orbital tensor): the cotangent of B from
// (Rbar_aa, Rbar_ab), then back through the pairwise contractions of B (the
// forward intermediates recomputed), the trace Y, the sigma weighting and the
// 2-cumulant to X, the 2-RDM and the 1-RDM, over n = 2r spin orbitals: 3
// forward and 12 backward n^2 x n^2 x n^2 GEMMs (FP64, or int8 exact-
// accumulation products under ACSE_INT8CRT), the rest in FP64.  The results are
// added to the Valdemoro adjoint's accumulators: Abaa, Abab (gradients of the
// fold's blocks), Gbaa, Gbab (half the gradients of d2aa, d2ab) and gbar (the
// 1-RDM's), before their projections.
acse_status ny_vjp_share_run(acse_ctx c, const acse_problem *p, const double *Aaa, const double *Aab,
                             const double *Rbar_aa, const double *Rbar_ab, double *Abaa, double *Abab,
                             double *Gbaa, double *Gbab, double *gbar) {
  const int r = p->r, n = 2 * r;
  const int64_t n2 = (int64_t)n * n, n3 = n2 * n;
  hipStream_t s = c->stream;
  const bool crt = c->crt_moduli != 0;  // block products on the int8 matrix cores
  StageTimer t6(c, 6);
  SoWs *wp = nullptr;
  acse_status st = ensure_so_ws(c, n, 12, wp);
  if (st != ACSE_OK) return st;
  SoWs &w = *wp;
  double *X = w.a[0], *C2 = w.a[1], *CS = w.a[2], *W1 = w.a[3], *M2 = w.a[4], *M3 = w.a[5];
  double *Bb = w.a[6], *Tb = w.a[7], *Wb = w.a[8], *Xb = w.a[9], *C2b = w.a[10], *CSb = w.a[11];
  std::vector<double> sig(c->ny_sigma);  // both spins of an orbital share its occupation
  sig.insert(sig.end(), c->ny_sigma.begin(), c->ny_sigma.end());
  if ((st = so_upload_sigma(c, w, sig)) != ACSE_OK) return st;
  // forward: X, the cumulants, the three first-stage intermediates, Y
  HIP_TRY(c, launch_so_embed_singlet_x(r, Aaa, Aab, X, s));
  HIP_TRY(c, launch_so_cumulant(r, p->d1, p->d1, p->d2aa, p->d2aa, p->d2ab, w.sig, C2, CS, s));
  if ((st = so_contract(c, w, n, W1, "kpia", X, "kprq", 1, C2, "iarq", 1, 1.0, 0, crt)) != ACSE_OK) return st;
  HIP_TRY(c, launch_so_trace_y(n, W1, w.Y, s));
  if ((st = so_contract(c, w, n, M2, "kqja", X, "kprq", 1, CS, "jpar", 1, 1.0, 0, crt)) != ACSE_OK) return st;
  if ((st = so_contract(c, w, n, M3, "kral", X, "kprq", 1, C2, "palq", 1, 1.0, 0, crt)) != ACSE_OK) return st;
  // cotangent of B; Tb = sw(Bbar), the cotangent shape of the sw() terms
  HIP_TRY(c, launch_so_bbar(r, Rbar_aa, Rbar_ab, 1.0, Bb, s));
  {
    Terms4 Q{};
    Q.n = 2;
    Q.t[0] = so_term(Bb, 1.0, n3, n2, n, 1);
    Q.t[1] = so_term(Bb, -1.0, n2, n3, n, 1);
    HIP_TRY(c, launch_combine4(n, Q, Tb, 0, nullptr, s));
  }
  // t_il (weight 4 on sw) and t_pl (weight 4, through Y)
  if ((st = so_contract(c, w, n, Wb, "kpia", Tb, "ijkl", 1, CS, "jpal", 1, 4.0, 0, crt)) != ACSE_OK) return st;
  HIP_TRY(c, launch_so_ybar(n, 4.0, Bb, CS, w.part, w.Yb, s));
  HIP_TRY(c, launch_so_diag_add(n, w.Yb, Wb, s));
  if ((st = so_contract(c, w, n, CSb, "jpal", Tb, "ijkl", 1, W1, "kpia", 1, 4.0, 0, crt)) != ACSE_OK) return st;
  HIP_TRY(c, launch_so_csbar_pl(n, 4.0, Bb, w.Y, CSb, s));
  if ((st = so_contract(c, w, n, Xb, "kprq", Wb, "kpia", 1, C2, "iarq", 1, 1.0, 0, crt)) != ACSE_OK) return st;
  if ((st = so_contract(c, w, n, C2b, "iarq", Wb, "kpia", 1, X, "kprq", 1, 1.0, 0, crt)) != ACSE_OK) return st;
  // t_ir (weight -8 on sw)
  if ((st = so_contract(c, w, n, Wb, "kqja", Tb, "ijkl", 1, C2, "ialq", 1, -8.0, 0, crt)) != ACSE_OK) return st;
  if ((st = so_contract(c, w, n, C2b, "ialq", Tb, "ijkl", 1, M2, "kqja", 3, -8.0, 1, crt)) != ACSE_OK) return st;
  if ((st = so_contract(c, w, n, Xb, "kprq", Wb, "kqja", 3, CS, "jpar", 1, 1.0, 1, crt)) != ACSE_OK) return st;
  if ((st = so_contract(c, w, n, CSb, "jpar", Wb, "kqja", 3, X, "kprq", 1, 1.0, 1, crt)) != ACSE_OK) return st;
  // t_pr (weight -8)
  if ((st = so_contract(c, w, n, Wb, "kral", Bb, "ijkl", 1, CS, "ijar", 1, -8.0, 0, crt)) != ACSE_OK) return st;
  if ((st = so_contract(c, w, n, CSb, "ijar", Bb, "ijkl", 1, M3, "kral", 3, -8.0, 1, crt)) != ACSE_OK) return st;
  if ((st = so_contract(c, w, n, Xb, "kprq", Wb, "kral", 3, C2, "palq", 1, 1.0, 1, crt)) != ACSE_OK) return st;
  if ((st = so_contract(c, w, n, C2b, "palq", Wb, "kral", 3, X, "kprq", 1, 1.0, 1, crt)) != ACSE_OK) return st;
  // cs = sigma_a c2, c2 = 2D - (1D^1D)/2, then the singlet lifts
  HIP_TRY(c, launch_so_sigma_fold(n, w.sig, CSb, C2b, s));
  HIP_TRY(c, launch_so_d1bar_singlet(r, p->d1, C2b, gbar, s));
  HIP_TRY(c, launch_so_dbar_singlet(r, 0.5, C2b, Gbaa, Gbab, s));
  HIP_TRY(c, launch_so_xbar_singlet(r, Xb, Abaa, Abab, s));
  return ACSE_OK;
}

acse_status ny_vjp_share(acse_ctx c, const acse_problem *p, const double *Aaa, const double *Aab,
                         const double *Rbar_aa, const double *Rbar_ab, double *Abaa, double *Abab, double *Gbaa,
                         double *Gbab, double *gbar) {
  try {
    return ny_vjp_share_run(c, p, Aaa, Aab, Rbar_aa, Rbar_ab, Abaa, Abab, Gbaa, Gbab, gbar);
  } catch (const std::exception &e) {
    return fail(c, ACSE_ERR_NOMEM, std::string("NY adjoint: ") + e.what());
  }
}

}  // namespace

extern "C" acse_status acse_residual_vjp(acse_ctx ctx, const acse_problem *prob,
                                         const acse_options *opts, const double *Rbar_aa,
                                         const double *Rbar_ab, double *h_bar, double *V_bar,
                                         double *d1_bar, double *d2aa_bar, double *d2ab_bar) {
  acse_status st = validate(ctx, prob, opts);
  if (st != ACSE_OK) return st;
  if (ctx->ny_on && prob->r > kSoMaxR)
    return fail(ctx, ACSE_ERR_UNSUPPORTED, "the NY adjoint runs up to r = " + std::to_string(kSoMaxR));
  for (const void *q : {static_cast<const void *>(Rbar_aa), static_cast<const void *>(Rbar_ab),
                        static_cast<const void *>(h_bar), static_cast<const void *>(V_bar),
                        static_cast<const void *>(d1_bar), static_cast<const void *>(d2aa_bar),
                        static_cast<const void *>(d2ab_bar)})
    if ((st = check_out(ctx, q, "VJP array")) != ACSE_OK) return st;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if ((st = ensure_vjp_ws(ctx)) != ACSE_OK) return st;
  // int8 exact accumulation: every operand is built in FP64 and converted to
  // residues before its grouped launch
  const bool crt = ctx->crt_moduli != 0;
  if (crt && (st = ensure_vjp_crt(ctx)) != ACSE_OK) return st;

  const int r = prob->r;
  const int N = prob->n_alpha + prob->n_beta;
  const int64_t r2 = (int64_t)r * r, r3 = r2 * r;
  const int ld = (int)op_ld(r);
  const int64_t Mp = op_rows(r);
  const GemmPrec prec = crt ? GEMM_F64 : prec_of(opts);
  const double *g = prob->d1;
  Workspace &w = ctx->ws;
  hipStream_t s = ctx->stream;
  const Nat4 nat(r);
  double **V = ctx->vnat;
  double *gb = ctx->vsmall, *tb = gb + r2, *fb = tb + r2, *Id = fb + r2, *hb_raw = Id + r2;
  // operand buffers of the adjoint GEMMs
  auto vop = [&](int q) {
    OperandRef o{ctx->vop[q], nullptr};
    if (prec == GEMM_BF16X3) o.lo = ctx->vop[q] + Mp * ld * 2;
    return o;
  };
  // natural r^4 destination
  auto natref = [&](double *p) { return OperandRef{p, nullptr}; };
  // The backward pass queues its permutes and launches the queue in batches
  // (launch_permute4_batch): before any other kernel, and before a permute
  // that would write what a queued one reads or writes, or read what one writes.
  PermArgs pq_a[kMaxPermJobs];
  OperandRef pq_o[kMaxPermJobs];
  GemmPrec pq_p[kMaxPermJobs];
  int pq_n = 0;
  auto flushq = [&]() -> hipError_t {
    if (!pq_n) return hipSuccess;
    const int n = pq_n;
    pq_n = 0;
    return launch_permute4_batch(pq_p, pq_a, pq_o, n, s);
  };
  const int64_t nat_bytes = r2 * r2 * 8;
  auto overlap = [](const void *p, int64_t pb, const void *q, int64_t qb) {
    if (!p || !q) return false;
    const char *x = static_cast<const char *>(p), *y = static_cast<const char *>(q);
    return x < y + qb && y < x + pb;
  };
  auto permute = [&](GemmPrec pr, const OperandRef &dst, bool operand_layout, const double *s1,
                     const int m1[4], double c1, const double *s2, const int m2[4], double c2,
                     int acc) -> hipError_t {
    PermArgs a{};
    a.r = r;
    a.rows = operand_layout ? Mp : r2;
    a.ld = operand_layout ? ld : r2;
    a.src1 = s1;
    nat.map(m1, a.s1);
    a.c1 = c1;
    a.src2 = s2;
    if (s2) nat.map(m2, a.s2);
    a.c2 = c2;
    a.accumulate = acc;
    const int64_t db = a.rows * a.ld * 8;
    bool clash = pq_n == kMaxPermJobs;
    for (int q = 0; q < pq_n && !clash; ++q) {
      const int64_t qb = pq_a[q].rows * pq_a[q].ld * 8;
      clash = overlap(dst.hi, db, pq_o[q].hi, qb) || overlap(dst.hi, db, pq_a[q].src1, nat_bytes) ||
              overlap(dst.hi, db, pq_a[q].src2, nat_bytes) || overlap(s1, nat_bytes, pq_o[q].hi, qb) ||
              overlap(s2, nat_bytes, pq_o[q].hi, qb);
    }
    if (clash) {
      hipError_t e = flushq();
      if (e != hipSuccess) return e;
    }
    pq_a[pq_n] = a;
    pq_o[pq_n] = dst;
    pq_p[pq_n] = pr;
    ++pq_n;
    return hipSuccess;
  };
  const int ID[4] = {0, 1, 2, 3};
  auto mode = [&](const double *in1, const double *in2, double c2, const double *M, int tr,
                  int64_t A, int64_t Bn, double alpha, double *out, int64_t adiv, int64_t so1,
                  int64_t so0, int64_t sx, int64_t sb, int cols_fast, int acc) -> hipError_t {
    hipError_t fe = flushq();
    if (fe != hipSuccess) return fe;
    ModeArgs m = mode_base(ctx, r, M);
    m.A = A; m.Bn = Bn; m.in1 = in1; m.in2 = in2; m.c2 = c2; m.transpose_m = tr;
    m.alpha = alpha; m.adiv = adiv; m.so1 = so1; m.so0 = so0; m.sx = sx; m.sb = sb;
    m.out_cols_fast = cols_fast; m.accumulate = acc;
    return launch_mode(GEMM_F64, m, OperandRef{out, nullptr}, s);
  };
  auto term = [&](const double *T, int px, int py, int pu, int pv, const double *M, double c) {
    ContractTerm t{};
    t.T = T; t.sx = nat.S[px]; t.sy = nat.S[py]; t.su = nat.S[pu]; t.sv = nat.S[pv]; t.M = M; t.c = c;
    return t;
  };
  auto contract = [&](std::initializer_list<ContractTerm> terms, double *out, int acc) -> hipError_t {
    hipError_t fe = flushq();
    if (fe != hipSuccess) return fe;
    ContractArgs a{};
    for (const ContractTerm &t : terms) a.term[a.nterms++] = t;
    return launch_contract42(r, a, out, acc, w.tpart, s);
  };

  // ---------------- forward recompute (natural layouts) -------------------
  HIP_TRY(ctx, flushq());
  if ((st = prep_rdm_operands(ctx, prob, prec)) != ACSE_OK) return st;
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_fold(r, N, prob->h, prob->V, w.Aaa, w.Aab, s));
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_f(r, w.Aaa, w.Aab, g, w.fpart, w.f, s));
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_t(r, w.Waa, w.Aaa, w.Wab, w.Aab, w.tpart, w.t, s, ctx->general));
  for (int b = 0; b < 2; ++b)
    HIP_TRY(ctx, mode(b ? w.Aab : w.Aaa, nullptr, 0.0, g, 1, r, r2, 1.0, b ? w.Hab : w.Haa, 1, r3, 0,
                      r2, 1, 1, 0));
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_g2(prec, r, ctx->general, w.Aaa, w.Aab, w.Haa, w.Hab, w.f, w.G2aa, w.G2ab, vop(0),
                         vop(1), vop(2), s));
  // B = A - G2, L+-, L3 and R+-, R3 are written straight into the GEMM operand
  // layouts where the products below need them.

  // ---------------- backward ----------------------------------------------
  double *Sbaa = V[8], *Sbab = V[9], *Ppb = V[10], *Pmb = V[11], *E3b = V[12];
  double *Lpb = V[13], *Lmb = V[14], *L3b = V[15], *Rpb = V[16], *Rmb = V[17], *R3b = V[18];
  double *Gbaa = V[19], *Gbab = V[20], *Bbaa = V[21], *Bbab = V[22], *Maa = V[23], *Mab = V[24];
  double *G2baa = V[25], *G2bab = V[26], *Abaa = V[27], *Abab = V[28], *Wbaa = V[29], *Wbab = V[30];
  double *T1 = V[31], *T2 = V[32], *T3 = V[33], *T4 = V[34], *Vraw = V[35];
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_fill(r2, 0.0, gb, s));
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_identity(r, Id, s));
  // S-bar = R-bar - R-bar^T  (R = S - S^T)
  {
    const int tr[4] = {2, 3, 0, 1};
    HIP_TRY(ctx, permute(GEMM_F64, natref(Sbaa), false, Rbar_aa, ID, 1.0, Rbar_aa, tr, -1.0, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(Sbab), false, Rbar_ab, ID, 1.0, Rbar_ab, tr, -1.0, 0));
  }
  // gamma-t terms: t-bar and gamma-bar (S_aa carries -gt_aa, S_ab carries +gt_ab)
  HIP_TRY(ctx, contract({term(Sbaa, 1, 2, 0, 3, g, -1.0), term(Sbaa, 0, 2, 1, 3, g, 1.0),
                         term(Sbaa, 1, 3, 0, 2, g, 1.0), term(Sbaa, 0, 3, 1, 2, g, -1.0),
                         term(Sbab, 0, 2, 1, 3, g, 1.0), term(Sbab, 1, 3, 0, 2, g, 1.0)},
                        tb, 0));
  HIP_TRY(ctx, contract({term(Sbaa, 0, 3, 1, 2, w.t, -1.0), term(Sbaa, 1, 3, 0, 2, w.t, 1.0),
                         term(Sbaa, 0, 2, 1, 3, w.t, 1.0), term(Sbaa, 1, 2, 0, 3, w.t, -1.0),
                         term(Sbab, 1, 3, 0, 2, w.t, 1.0), term(Sbab, 0, 2, 1, 3, w.t, 1.0)},
                        gb, 1));
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_vjp_pe(r, Sbaa, Sbab, Ppb, Pmb, E3b, s));

  int kdim[kMaxGemmProbs] = {};  // K of each product of the batch being built
  auto gemm_set = [&](GemmBatch &b, int q, int ia, int ib, double alpha, double *C, const int om[4]) {
    GemmProb &P = b.p[q];
    kdim[q] = (int)r2;
    OperandRef a = vop(ia), bb = vop(ib);
    P.A = a.hi; P.A2 = a.lo; P.B = bb.hi; P.B2 = bb.lo;
    P.C = C; P.alpha = alpha;
    P.M = (int)r2; P.N = (int)r2; P.Kp = gemm_kp(prec, (int)r2, ld); P.ld = ld; P.rdiv = r;
    // output (m/r, m%r, n/r, n%r) -> natural positions om[0..3] of the result
    P.sm1 = nat.S[om[0]]; P.sm0 = nat.S[om[1]]; P.sn1 = nat.S[om[2]]; P.sn0 = nat.S[om[3]];
    P.ksplit = 1; P.kchunk = P.Kp; P.accumulate = 0;
  };
  int use_cfg = opts ? opts->tile : -1;
  if (use_cfg < 0) {
    auto it = ctx->tuned.find({r, (int)prec});
    use_cfg = it != ctx->tuned.end() ? it->second : gemm_default_cfg(prec, (int)r2, (int)r2);
  }
  // one grouped launch of adjoint products: on the tiles of the call's
  // precision, or (int8 exact accumulation) the residues of every operand
  // buffer the batch reads, the modular products (reconstruction factors in
  // their epilogue) and the reconstruction through the same store maps
  auto vop_index = [&](const void *p) {
    for (int q = 0; q < 12; ++q)
      if (ctx->vop[q] == p) return q;
    return -1;
  };
  auto vjp_gemm = [&](GemmBatch &b) -> acse_status {
    HIP_TRY(ctx, flushq());
    if (!crt) {
      HIP_TRY(ctx, flushq());
      HIP_TRY(ctx, gemm_launch(prec, use_cfg, b, s));
      return ACSE_OK;
    }
    int bk[12] = {}, brows[12] = {}, bld[12] = {};
    int ia[kMaxGemmProbs] = {}, ib[kMaxGemmProbs] = {};
    for (int k = 0; k < b.count; ++k) {
      const GemmProb &P = b.p[k];
      ia[k] = vop_index(P.A);
      ib[k] = vop_index(P.B);
      if (ia[k] < 0 || ib[k] < 0) return fail(ctx, ACSE_ERR_HIP, "adjoint product operand outside its buffers");
      for (int side = 0; side < 2; ++side) {
        const int q = side ? ib[k] : ia[k];
        if (bk[q] && bk[q] != kdim[k]) return fail(ctx, ACSE_ERR_HIP, "adjoint operand buffer read with two K");
        bk[q] = kdim[k];
        bld[q] = P.ld;
        brows[q] = std::max(brows[q], side ? P.N : P.M);
      }
    }
    ResidueBatch rb{};
    int nrows = 0;
    for (int q = 0; q < 12; ++q) {
      if (!bk[q]) continue;
      ResidueJob &J = rb.job[rb.count++];
      J.src = reinterpret_cast<const double *>(ctx->vop[q]);
      J.dst = ctx->vcres[q];
      J.e = ctx->vcexp[q];
      J.plane = Mp * crt_ldr(bk[q]);
      J.row_begin = nrows;
      J.K = bk[q];
      J.ld = bld[q];
      J.ldr = (int)crt_ldr(bk[q]);
      J.kbits = crt_kbits(ctx->crt, bk[q]);
      J.premul = 0;
      nrows += brows[q];
    }
    rb.total_rows = nrows;
    HIP_TRY(ctx, flushq());
    HIP_TRY(ctx, launch_to_residues(rb, ctx->crt, s));
    int64_t yoff = 0;  // the products' residues one after another (their sizes differ)
    for (int k = 0; k < b.count; ++k) {
      GemmProb &G = b.p[k];
      const int K = kdim[k];
      G.A = ctx->vcres[ia[k]];
      G.B = ctx->vcres[ib[k]];
      G.A2 = G.B2 = nullptr;
      G.ld = G.Kp = (int)crt_ldr(K);
      G.kchunk = G.Kp;
      G.plane_a = G.plane_b = Mp * crt_ldr(K);
      G.ea = ctx->vcexp[ia[k]];
      G.eb = ctx->vcexp[ib[k]];
      G.kshift = 2 * crt_kbits(ctx->crt, K);
      G.u_out = 1;
      G.plane_y = crt_residue_out_bytes(G.M, G.N);
      G.Y = ctx->vcy + yoff;
      yoff += (int64_t)ctx->crt.nmod * G.plane_y;
    }
    HIP_TRY(ctx, flushq());
    HIP_TRY(ctx, gemm_crt_launch(b, ctx->crt, s));
    HIP_TRY(ctx, crt_combine_launch(b, ctx->crt, s));
    return ACSE_OK;
  };
  {  // particle-hole adjoint products
    // L+b[(k,i),(p,s)] = sum_(j,l) P+b[i,j,k,l] R+[j,l,p,s];  R+b[(j,l),(p,s)] = sum_(k,i) P+b L+[k,i,p,s]
    const int Akijl[4] = {2, 0, 1, 3}, Ajlki[4] = {1, 3, 2, 0};
    const int Akjil[4] = {2, 1, 0, 3}, Ailkj[4] = {0, 3, 2, 1};
    // R+-[j,l,p,s] = W_aa[j,p,s,l] -+ W_ab[j,p,l,s], R3[i,l,p,s] = W_ab[i,p,s,l], as rows (p,s), cols (j,l)
    const int Rwaa[4] = {1, 2, 0, 3}, Rwab[4] = {1, 3, 0, 2};
    // L+-[k,i,p,s] = sum_r g[i,r] (A_aa +- A_ab)[k,p,r,s], L3[k,j,p,s] = sum_r g[j,r] A_ab[k,p,s,r],
    // as rows (p,s), cols (k,i): written by the mode products with operand strides
    auto lop = [&](int q, const double *in1, const double *in2, double c2, int64_t A, int64_t Bn,
                   int64_t adiv, int64_t so1, int64_t so0, int64_t sb) -> hipError_t {
      hipError_t e = flushq();
      if (e != hipSuccess) return e;
      e = launch_zero_kpad(prec, r, ld, vop(q), s);
      if (e != hipSuccess) return e;
      ModeArgs m = mode_base(ctx, r, g);
      m.A = A; m.Bn = Bn; m.in1 = in1; m.in2 = in2; m.c2 = c2;
      m.adiv = adiv; m.so1 = so1; m.so0 = so0; m.sx = 1; m.sb = sb; m.out_cols_fast = 1;
      return launch_mode(prec, m, vop(q), s);
    };
    HIP_TRY(ctx, permute(prec, vop(0), true, Ppb, Akijl, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, permute(prec, vop(1), true, w.Waa, Rwaa, 1.0, w.Wab, Rwab, -1.0, 0));
    HIP_TRY(ctx, permute(prec, vop(2), true, Ppb, Ajlki, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, lop(3, w.Aaa, w.Aab, 1.0, r2, r, r, r, (int64_t)r * ld, ld));
    HIP_TRY(ctx, permute(prec, vop(4), true, Pmb, Akijl, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, permute(prec, vop(5), true, w.Waa, Rwaa, 1.0, w.Wab, Rwab, 1.0, 0));
    HIP_TRY(ctx, permute(prec, vop(6), true, Pmb, Ajlki, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, lop(7, w.Aaa, w.Aab, -1.0, r2, r, r, r, (int64_t)r * ld, ld));
    // L3b[(k,j),(p,s)] = -2 sum_(i,l) E3b[i,j,k,l] R3[i,l,p,s];  R3b[(i,l),(p,s)] = -2 sum_(k,j) E3b L3[k,j,p,s]
    HIP_TRY(ctx, permute(prec, vop(8), true, E3b, Akjil, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, permute(prec, vop(9), true, w.Wab, Rwaa, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, permute(prec, vop(10), true, E3b, Ailkj, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, lop(11, w.Aab, nullptr, 0.0, r3, 1, r2, r, ld, 0));

    GemmBatch b{};
    b.count = 6;
    gemm_set(b, 0, 0, 1, 1.0, Lpb, ID);
    gemm_set(b, 1, 2, 3, 1.0, Rpb, ID);
    gemm_set(b, 2, 4, 5, 1.0, Lmb, ID);
    gemm_set(b, 3, 6, 7, 1.0, Rmb, ID);
    gemm_set(b, 4, 8, 9, -2.0, L3b, ID);
    gemm_set(b, 5, 10, 11, -2.0, R3b, ID);
    if ((st = vjp_gemm(b)) != ACSE_OK) return st;
  }
  {  // particle-particle adjoint products
    // G-bar = Z-bar B^T-products:  Gb[(ij),(rs)] = sum_(kl) Sb[ij,kl] B[kl,rs]
    //                              Bb[(kl),(rs)] = sum_(ij) Sb[ij,kl] Gamma2[ij,rs]
    //                              M[(ij),(rs)]  = sum_(kl) Sb[ij,kl] G2[kl,rs]
    // all packed over the pair symmetries of Gamma2, B and G2 (pairs (a<b) or
    // (a<=b) in packing order; Gamma2_aa = 2 d2aa, Gamma2_ab = 2 d2ab):
    //  alpha-alpha (Gamma2, B, G2 antisymmetric within both pairs):
    //   Gb_aa enters only through its projection onto that subspace, whose value is
    //     1/2 sum_(k<l) ZAA[(i<j),(k<l)] B[(k<l),(r<s)],  ZAA = Sb - Sb(i<->j) - Sb(k<->l) + Sb(both);
    //   Bb_aa[(kl),(r<s)] = 2 sum_(i<j) (Sb[ij,kl] - Sb[ji,kl]) Gamma2_aa[ij,rs];
    //   M_aa[(ij),(r<s)]  = sum_(k<l) (Sb[ij,kl] - Sb[ij,lk]) G2_aa[kl,rs].
    //  alpha-beta (Gamma2, B, G2 invariant under (ij)(kl) -> (ji)(lk)): each
    //  product splits by r <-> s into X+- = X[.,rs] +- X[.,sr], X = (X+ + X-)/2,
    //  with the summed pair packed as k <= l (+) and k < l (-):
    //   Gb_ab enters only through its projection onto that symmetry, whose value
    //     is 2 Zt B with Zt = (Sb + Sb[ji,lk]) / 2; its + part is symmetric and
    //     its - part antisymmetric in (i,j), so rows are packed too;
    //   Bb_ab+- = 2 sum_(i<=j / i<j) (Sb[ij,kl] +- Sb[ji,kl]) Gamma2_ab+-[ij,rs] (i = j once);
    //   M_ab+-  = sum_(k<=l / k<l) (Sb[ij,kl] +- Sb[ij,lk]) G2_ab+-[kl,rs] (k = l once).
    const int nlt = npair_lt(r), nle = npair_le(r);
    const int64_t ldlt = ld_pair_lt(r), ldle = ld_pair_le(r);
    struct PackTerm { const double *src; const int *map; double c; int offdiag; };
    auto pack = [&](int q, int rows_mode, int k_le, std::initializer_list<PackTerm> terms) -> hipError_t {
      hipError_t fe = flushq();
      if (fe != hipSuccess) return fe;
      PairPackArgs a{};
      a.r = r;
      a.rows_mode = rows_mode;
      a.k_le = k_le;
      a.ld = k_le ? ldle : ldlt;
      for (const PackTerm &t : terms) {
        a.src[a.nterms] = t.src;
        nat.map(t.map, a.st[a.nterms]);
        a.c[a.nterms] = t.c;
        a.offdiag[a.nterms] = t.offdiag;
        ++a.nterms;
      }
      return launch_pack_pairs(prec, a, vop(q), s);
    };
    // index maps: term X[...] of the letters (a,b) = packed row pair, (c,d) = packed K pair
    const int abcd[4] = {0, 1, 2, 3}, bacd[4] = {1, 0, 2, 3}, abdc[4] = {0, 1, 3, 2}, badc[4] = {1, 0, 3, 2};
    // packed products: C[m][n] = alpha sum_k A[m][k] B[n][k] into row-major [M][N] scratch
    auto pair_set = [&](GemmBatch &b, int q, int ia, int ib, double alpha, double *C, int M, int N, int k_le) {
      GemmProb &P = b.p[q];
      OperandRef a = vop(ia), bb = vop(ib);
      const int K = k_le ? nle : nlt, ldk = (int)(k_le ? ldle : ldlt);
      kdim[q] = K;
      P.A = a.hi; P.A2 = a.lo; P.B = bb.hi; P.B2 = bb.lo;
      P.C = C; P.alpha = alpha;
      P.M = M; P.N = N; P.Kp = gemm_kp(prec, K, ldk); P.ld = ldk; P.rdiv = 1;
      P.sm1 = N; P.sm0 = 0; P.sn1 = 1; P.sn0 = 0;
      P.ksplit = 1; P.kchunk = P.Kp; P.accumulate = 0;
    };
    // The packing passes read the summed pair along the fast source index: a
    // source whose summed pair is its leading pair is first exchanged
    // ((ij) <-> (kl), X^T[a,b,c,d] = X[c,d,a,b]) into a buffer that is free
    // until the products' results are unpacked.
    const int XT[4] = {2, 3, 0, 1};
    auto exch = [&](double *dst, const double *x, const double *y, double cy) -> hipError_t {
      return permute(GEMM_F64, natref(dst), false, x, XT, 1.0, y, XT, cy, 0);
    };
    auto pack_aa = [&]() -> hipError_t {
      double *SbaaT = Gbaa, *BaaT = Bbaa, *G2aaT = Maa, *DaaT = Vraw;
      hipError_t e;
      if ((e = exch(SbaaT, Sbaa, nullptr, 0.0)) != hipSuccess) return e;
      if ((e = exch(BaaT, w.Aaa, w.G2aa, -1.0)) != hipSuccess) return e;
      if ((e = exch(G2aaT, w.G2aa, nullptr, 0.0)) != hipSuccess) return e;
      if ((e = exch(DaaT, prob->d2aa, nullptr, 0.0)) != hipSuccess) return e;
      if ((e = pack(0, 1, 0, {{Sbaa, abcd, 1.0, 0}, {Sbaa, bacd, -1.0, 0}, {Sbaa, abdc, -1.0, 0},
                              {Sbaa, badc, 1.0, 0}})) != hipSuccess) return e;
      if ((e = pack(1, 1, 0, {{BaaT, abcd, 1.0, 0}})) != hipSuccess) return e;
      if ((e = pack(2, 0, 0, {{SbaaT, abcd, 1.0, 0}, {SbaaT, abdc, -1.0, 0}})) != hipSuccess) return e;
      if ((e = pack(3, 1, 0, {{DaaT, abcd, 1.0, 0}})) != hipSuccess) return e;
      if ((e = pack(4, 0, 0, {{Sbaa, abcd, 1.0, 0}, {Sbaa, abdc, -1.0, 0}})) != hipSuccess) return e;
      return pack(5, 1, 0, {{G2aaT, abcd, 1.0, 0}});
    };
    const int R2 = (int)r2;
    double *Gp = T4, *Gm = T4 + (int64_t)nle * nle;  // Gb_ab +- (rows packed)
    // Below kAbPackMinR the packing passes and the second launch cost more than
    // the alpha-beta flops they save: those products run unpacked there (the
    // general-kernel option takes the packed form at every r).
    const bool pack_ab = r >= kAbPackMinR || ctx->general;
    if (!pack_ab) {
      const int Akl_ij[4] = {2, 3, 0, 1};   // Sb[i,j,k,l] as rows (k,l), cols (i,j)
      const int Brs_kl[4] = {2, 3, 0, 1};   // X[k,l,r,s] as rows (r,s), cols (k,l)
      HIP_TRY(ctx, pack_aa());
      HIP_TRY(ctx, permute(prec, vop(6), true, Sbab, ID, 1.0, nullptr, ID, 0.0, 0));
      HIP_TRY(ctx, permute(prec, vop(7), true, Sbab, Akl_ij, 1.0, nullptr, ID, 0.0, 0));
      HIP_TRY(ctx, permute(prec, vop(8), true, w.Aab, Brs_kl, 1.0, w.G2ab, Brs_kl, -1.0, 0));
      HIP_TRY(ctx, permute(prec, vop(9), true, prob->d2ab, Brs_kl, 1.0, nullptr, ID, 0.0, 0));
      HIP_TRY(ctx, permute(prec, vop(10), true, w.G2ab, Brs_kl, 1.0, nullptr, ID, 0.0, 0));
      GemmBatch b{};
      b.count = 6;
      pair_set(b, 0, 0, 1, 0.5, T1, nlt, nlt, 0);
      pair_set(b, 1, 2, 3, 2.0, T2, R2, nlt, 0);
      pair_set(b, 2, 4, 5, 1.0, T3, R2, nlt, 0);
      gemm_set(b, 3, 6, 8, 2.0, Gbab, ID);
      gemm_set(b, 4, 7, 9, 4.0, Bbab, ID);   // 2 * Gamma2_ab = 4 d2ab
      gemm_set(b, 5, 6, 10, 1.0, Mab, ID);
      if ((st = vjp_gemm(b)) != ACSE_OK) return st;
      HIP_TRY(ctx, flushq());
      HIP_TRY(ctx, launch_unpack_pairs(r, 1, T1, nlt, Gbaa, s));
      HIP_TRY(ctx, flushq());
      HIP_TRY(ctx, launch_unpack_pairs(r, 0, T2, nlt, Bbaa, s));
      HIP_TRY(ctx, flushq());
      HIP_TRY(ctx, launch_unpack_pairs(r, 0, T3, nlt, Maa, s));
    }
    if (pack_ab) {
      HIP_TRY(ctx, pack_aa());
      HIP_TRY(ctx, pack(6, 2, 1, {{Sbab, abcd, 0.5, 0}, {Sbab, badc, 0.5, 0}, {Sbab, abdc, 0.5, 1},
                                  {Sbab, bacd, 0.5, 1}}));
      double *BabT = Gbab;
      HIP_TRY(ctx, exch(BabT, w.Aab, w.G2ab, -1.0));
      HIP_TRY(ctx, pack(7, 2, 1, {{BabT, abcd, 1.0, 0}, {BabT, bacd, 1.0, 0}}));
      HIP_TRY(ctx, pack(8, 1, 0, {{Sbab, abcd, 0.5, 0}, {Sbab, badc, 0.5, 0}, {Sbab, abdc, -0.5, 0},
                                  {Sbab, bacd, -0.5, 0}}));
      HIP_TRY(ctx, pack(9, 1, 0, {{BabT, abcd, 1.0, 0}, {BabT, bacd, -1.0, 0}}));
      GemmBatch b{};
      b.count = 5;
      pair_set(b, 0, 0, 1, 0.5, T1, nlt, nlt, 0);
      pair_set(b, 1, 2, 3, 2.0, T2, R2, nlt, 0);
      pair_set(b, 2, 4, 5, 1.0, T3, R2, nlt, 0);
      pair_set(b, 3, 6, 7, 2.0, Gp, nle, nle, 1);
      pair_set(b, 4, 8, 9, 2.0, Gm, nlt, nlt, 0);
      if ((st = vjp_gemm(b)) != ACSE_OK) return st;
      HIP_TRY(ctx, flushq());
      HIP_TRY(ctx, launch_unpack_pairs(r, 1, T1, nlt, Gbaa, s));
      HIP_TRY(ctx, flushq());
      HIP_TRY(ctx, launch_unpack_pairs(r, 0, T2, nlt, Bbaa, s));
      HIP_TRY(ctx, flushq());
      HIP_TRY(ctx, launch_unpack_pairs(r, 0, T3, nlt, Maa, s));
      HIP_TRY(ctx, flushq());
      HIP_TRY(ctx, launch_unpack_pm(r, 1, Gp, nle, Gm, nlt, Gbab, s));
    }
    if (pack_ab) {
      double *Bp = T1, *Bm = T1 + (int64_t)r2 * nle, *Mp = T2, *Mm = T2 + (int64_t)r2 * nle;
      double *SbabT = T3, *DabT = T4, *G2abT = Vraw;
      HIP_TRY(ctx, exch(SbabT, Sbab, nullptr, 0.0));
      HIP_TRY(ctx, exch(DabT, prob->d2ab, nullptr, 0.0));
      HIP_TRY(ctx, exch(G2abT, w.G2ab, nullptr, 0.0));
      HIP_TRY(ctx, pack(0, 0, 1, {{SbabT, abcd, 1.0, 0}, {SbabT, abdc, 1.0, 1}}));
      HIP_TRY(ctx, pack(1, 2, 1, {{DabT, abcd, 1.0, 0}, {DabT, bacd, 1.0, 0}}));
      HIP_TRY(ctx, pack(2, 0, 0, {{SbabT, abcd, 1.0, 0}, {SbabT, abdc, -1.0, 0}}));
      HIP_TRY(ctx, pack(3, 1, 0, {{DabT, abcd, 1.0, 0}, {DabT, bacd, -1.0, 0}}));
      HIP_TRY(ctx, pack(4, 0, 1, {{Sbab, abcd, 1.0, 0}, {Sbab, abdc, 1.0, 1}}));
      HIP_TRY(ctx, pack(5, 2, 1, {{G2abT, abcd, 1.0, 0}, {G2abT, bacd, 1.0, 0}}));
      HIP_TRY(ctx, pack(6, 0, 0, {{Sbab, abcd, 1.0, 0}, {Sbab, abdc, -1.0, 0}}));
      HIP_TRY(ctx, pack(7, 1, 0, {{G2abT, abcd, 1.0, 0}, {G2abT, bacd, -1.0, 0}}));
      GemmBatch b{};
      b.count = 4;
      pair_set(b, 0, 0, 1, 4.0, Bp, R2, nle, 1);  // 2 Gamma2_ab = 4 d2ab
      pair_set(b, 1, 2, 3, 4.0, Bm, R2, nlt, 0);
      pair_set(b, 2, 4, 5, 1.0, Mp, R2, nle, 1);
      pair_set(b, 3, 6, 7, 1.0, Mm, R2, nlt, 0);
      if ((st = vjp_gemm(b)) != ACSE_OK) return st;
      HIP_TRY(ctx, flushq());
      HIP_TRY(ctx, launch_unpack_pm(r, 0, Bp, nle, Bm, nlt, Bbab, s));
      HIP_TRY(ctx, flushq());
      HIP_TRY(ctx, launch_unpack_pm(r, 0, Mp, nle, Mm, nlt, Mab, s));
    }
  }
  // G2-bar = 4/3 (gamma x gamma) S-bar^T - B-bar;  A-bar += B-bar
  {
    const int tr[4] = {2, 3, 0, 1};
    for (int b = 0; b < 2; ++b) {
      const double *Sb = b ? Sbab : Sbaa;
      double *G2b = b ? G2bab : G2baa;
      const double *Bb = b ? Bbab : Bbaa;
      double *Ab = b ? Abab : Abaa;
      HIP_TRY(ctx, permute(GEMM_F64, natref(T1), false, Sb, tr, 1.0, nullptr, ID, 0.0, 0));  // [k,l,i,j]
      // T2[k,l,i,s] = sum_j g[j,s] T1[k,l,i,j]
      HIP_TRY(ctx, mode(T1, nullptr, 0.0, g, 1, r3, 1, 1.0, T2, 1, r, 0, 1, 0, 0, 0));
      // G2b[k,l,r,s] = 4/3 sum_i g[i,r] T2[k,l,i,s]
      HIP_TRY(ctx, mode(T2, nullptr, 0.0, g, 1, r2, r, 4.0 / 3.0, G2b, 1, r2, 0, r, 1, 1, 0));
      HIP_TRY(ctx, permute(GEMM_F64, natref(G2b), false, Bb, ID, -1.0, nullptr, ID, 0.0, 1));
      HIP_TRY(ctx, permute(GEMM_F64, natref(Ab), false, Bb, ID, 1.0, nullptr, ID, 0.0, 0));
    }
  }
  // gamma-bar from M = S-bar G2:  4/3 (sum_js M[i,j,r,s] g[j,s] + sum_ir M[i,j,r,s] g[i,r])
  HIP_TRY(ctx, contract({term(Maa, 0, 2, 1, 3, g, 4.0 / 3.0), term(Maa, 1, 3, 0, 2, g, 4.0 / 3.0),
                         term(Mab, 0, 2, 1, 3, g, 4.0 / 3.0), term(Mab, 1, 3, 0, 2, g, 4.0 / 3.0)},
                        gb, 1));
  // H-bar and f-bar from G2-bar
  {
    const int lk_aa[4] = {1, 0, 2, 3}, lk_ab[4] = {1, 0, 3, 2};
    HIP_TRY(ctx, permute(GEMM_F64, natref(Ppb), false, G2baa, ID, 1.0, G2baa, lk_aa, -1.0, 0));  // Hbaa
    HIP_TRY(ctx, permute(GEMM_F64, natref(Pmb), false, G2bab, ID, 1.0, G2bab, lk_ab, 1.0, 0));   // Hbab
  }
  double *Hbaa = Ppb, *Hbab = Pmb;
  HIP_TRY(ctx, contract({term(G2baa, 0, 2, 1, 3, Id, 1.0), term(G2baa, 0, 3, 1, 2, Id, -1.0),
                         term(G2baa, 1, 2, 0, 3, Id, -1.0), term(G2baa, 1, 3, 0, 2, Id, 1.0),
                         term(G2bab, 0, 2, 1, 3, Id, 1.0), term(G2bab, 1, 3, 0, 2, Id, 1.0)},
                        fb, 0));
  // H = A g: A-bar[k,p,(rs)] += sum_l g[p,l] H-bar[k,l,(rs)];  g-bar[p,l] += sum A[k,p,r,s] H-bar[k,l,r,s]
  for (int b = 0; b < 2; ++b)
    HIP_TRY(ctx, mode(b ? Hbab : Hbaa, nullptr, 0.0, g, 0, r, r2, 1.0, b ? Abab : Abaa, 1, r3, 0, r2, 1, 1, 1));
  {
    const int lead1[4] = {1, 0, 2, 3};   // [p][k,r,s] from X[k,p,r,s]
    HIP_TRY(ctx, permute(GEMM_F64, natref(T1), false, w.Aaa, lead1, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(T2), false, Hbaa, lead1, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(T3), false, w.Aab, lead1, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(T4), false, Hbab, lead1, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, flushq());
    HIP_TRY(ctx, launch_gram(r, T1, T2, 1.0, T3, T4, 1.0, w.tpart, gb, 1, s, ctx->general));
  }
  // W-bar from the ph B operands
  {
    const int waa[4] = {0, 2, 3, 1};   // W_aa[j,p,s,l] <- R[j,l,p,s]
    const int wab[4] = {0, 2, 1, 3};   // W_ab[j,p,l,s] <- R[j,l,p,s]
    HIP_TRY(ctx, permute(GEMM_F64, natref(Wbaa), false, Rpb, waa, 1.0, Rmb, waa, 1.0, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(Wbab), false, Rmb, wab, 1.0, Rpb, wab, -1.0, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(Wbab), false, R3b, waa, 1.0, nullptr, ID, 0.0, 1));
  }
  // t = W A^T:  W-bar[j,(prs)] += sum_k t-bar[j,k] A[k,(prs)];  A-bar[k,(prs)] += sum_j t-bar[j,k] W[j,(prs)]
  HIP_TRY(ctx, mode(w.Aaa, nullptr, 0.0, tb, 0, 1, r3, 1.0, Wbaa, 1, 0, 0, r3, 1, 1, 1));
  HIP_TRY(ctx, mode(w.Aab, nullptr, 0.0, tb, 0, 1, r3, 2.0, Wbab, 1, 0, 0, r3, 1, 1, 1));
  HIP_TRY(ctx, mode(w.Waa, nullptr, 0.0, tb, 1, 1, r3, 1.0, Abaa, 1, 0, 0, r3, 1, 1, 1));
  HIP_TRY(ctx, mode(w.Wab, nullptr, 0.0, tb, 1, 1, r3, 2.0, Abab, 1, 0, 0, r3, 1, 1, 1));
  // f terms
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_vjp_frank(r, fb, g, Abaa, Abab, s));
  HIP_TRY(ctx, contract({term(w.Aaa, 1, 2, 0, 3, fb, 1.0), term(w.Aab, 1, 3, 0, 2, fb, -1.0)}, gb, 1));
  // L terms: A-bar[k,p,r,s] += sum_i g[i,r] (L+b +- L-b)[k,i,p,s]; L3: A_ab-bar[k,p,s,r] += sum_j g[j,r] L3b[k,j,p,s]
  {
    const int kprs_from_krps[4] = {0, 2, 1, 3};   // dst (k,p,r,s) <- T[k,r,p,s]
    const int kpsr_from_krps[4] = {0, 2, 3, 1};   // dst (k,p,s,r) <- T[k,r,p,s]
    HIP_TRY(ctx, mode(Lpb, Lmb, 1.0, g, 1, r, r2, 1.0, T1, 1, r3, 0, r2, 1, 1, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(Abaa), false, T1, kprs_from_krps, 1.0, nullptr, ID, 0.0, 1));
    HIP_TRY(ctx, mode(Lpb, Lmb, -1.0, g, 1, r, r2, 1.0, T1, 1, r3, 0, r2, 1, 1, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(Abab), false, T1, kprs_from_krps, 1.0, nullptr, ID, 0.0, 1));
    HIP_TRY(ctx, mode(L3b, nullptr, 0.0, g, 1, r, r2, 1.0, T1, 1, r3, 0, r2, 1, 1, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(Abab), false, T1, kpsr_from_krps, 1.0, nullptr, ID, 0.0, 1));
    // gamma-bar[i,r] += sum L+b[k,i,p,s] (A_aa + A_ab)[k,p,r,s] + L-b (A_aa - A_ab)
    const int i_kps[4] = {1, 0, 2, 3};   // [i][k,p,s] from L[k,i,p,s]
    const int r_kps[4] = {2, 0, 1, 3};   // [r][k,p,s] from X[k,p,r,s]
    HIP_TRY(ctx, permute(GEMM_F64, natref(T1), false, Lpb, i_kps, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(T2), false, w.Aaa, r_kps, 1.0, w.Aab, r_kps, 1.0, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(T3), false, Lmb, i_kps, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(T4), false, w.Aaa, r_kps, 1.0, w.Aab, r_kps, -1.0, 0));
    HIP_TRY(ctx, flushq());
    HIP_TRY(ctx, launch_gram(r, T1, T2, 1.0, T3, T4, 1.0, w.tpart, gb, 1, s, ctx->general));
    // gamma-bar[j,r] += sum L3b[k,j,p,s] A_ab[k,p,s,r]
    const int r_kps3[4] = {3, 0, 1, 2};  // [r][k,p,s] from A_ab[k,p,s,r]
    HIP_TRY(ctx, permute(GEMM_F64, natref(T1), false, L3b, i_kps, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, permute(GEMM_F64, natref(T2), false, w.Aab, r_kps3, 1.0, nullptr, ID, 0.0, 0));
    HIP_TRY(ctx, flushq());
    HIP_TRY(ctx, launch_gram(r, T1, T2, 1.0, nullptr, nullptr, 0.0, w.tpart, gb, 1, s, ctx->general));
  }
  // W = Gamma2 - 2/3 g^g:  gamma-bar from W-bar
  HIP_TRY(ctx, contract({term(Wbaa, 0, 2, 1, 3, g, -2.0 / 3.0), term(Wbaa, 1, 3, 0, 2, g, -2.0 / 3.0),
                         term(Wbaa, 0, 3, 1, 2, g, 2.0 / 3.0), term(Wbaa, 1, 2, 0, 3, g, 2.0 / 3.0),
                         term(Wbab, 0, 2, 1, 3, g, -2.0 / 3.0), term(Wbab, 1, 3, 0, 2, g, -2.0 / 3.0)},
                        gb, 1));
  // the NY share's adjoint joins the accumulators before their projections
  HIP_TRY(ctx, flushq());
  if (ctx->ny_on && (st = ny_vjp_share(ctx, prob, w.Aaa, w.Aab, Rbar_aa, Rbar_ab, Abaa, Abab, Gbaa, Gbab, gb)) !=
                        ACSE_OK)
    return st;
  // Gamma2-bar = G-bar (GEMM) + W-bar;  d2-bar = 2 Gamma2-bar (projected)
  HIP_TRY(ctx, permute(GEMM_F64, natref(Gbaa), false, Wbaa, ID, 1.0, nullptr, ID, 0.0, 1));
  HIP_TRY(ctx, permute(GEMM_F64, natref(Gbab), false, Wbab, ID, 1.0, nullptr, ID, 0.0, 1));
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_proj(PROJ_AA, r, 2.0, Gbaa, d2aa_bar, s));
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_proj(PROJ_AB, r, 2.0, Gbab, d2ab_bar, s));
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_proj(PROJ_SYM2, r, 1.0, gb, d1_bar, s));
  // fold adjoint -> V-bar, h-bar
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_vjp_fold(r, N, Abaa, Abab, Vraw, hb_raw, s));
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_proj(PROJ_V, r, 1.0, Vraw, V_bar, s));
  HIP_TRY(ctx, flushq());
  HIP_TRY(ctx, launch_proj(PROJ_SYM2, r, 1.0, hb_raw, h_bar, s));
  HIP_TRY(ctx, flushq());
  return ACSE_OK;
}

extern "C" acse_status acse_energy_vjp(acse_ctx ctx, const acse_problem *prob, double Ebar,
                                       double *h_bar, double *V_bar, double *d2aa_bar,
                                       double *d2ab_bar) {
  acse_status st = validate(ctx, prob, nullptr, false);
  if (st != ACSE_OK) return st;
  if (!std::isfinite(Ebar)) return fail(ctx, ACSE_ERR_ARG, "Ebar is not finite");
  for (const void *q : {static_cast<const void *>(h_bar), static_cast<const void *>(V_bar),
                        static_cast<const void *>(d2aa_bar), static_cast<const void *>(d2ab_bar)})
    if ((st = check_out(ctx, q, "VJP array")) != ACSE_OK) return st;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if ((st = ensure_vjp_ws(ctx)) != ACSE_OK) return st;
  const int r = prob->r;
  const int N = prob->n_alpha + prob->n_beta;
  const int64_t r2 = (int64_t)r * r;
  Workspace &w = ctx->ws;
  hipStream_t s = ctx->stream;
  double *zero = ctx->vnat[0], *D = ctx->vnat[1], *Vraw = ctx->vnat[2];
  double *hb_raw = ctx->vsmall + 4 * r2;
  // E = 2 <K_s, d2aa + d2ab> with K_s = 2 A_ab of the fold:
  //   d2-bar = 2 Ebar K_s (projected);  through the fold, K_s-bar = 2 Ebar (d2aa + d2ab)
  HIP_TRY(ctx, launch_fold(r, N, prob->h, prob->V, w.Aaa, w.Aab, s));
  HIP_TRY(ctx, launch_proj(PROJ_AA, r, 4.0 * Ebar, w.Aab, d2aa_bar, s));
  HIP_TRY(ctx, launch_proj(PROJ_AB, r, 4.0 * Ebar, w.Aab, d2ab_bar, s));
  PermArgs a{};
  a.r = r; a.rows = r2; a.ld = r2;
  a.src1 = prob->d2aa; a.s1[0] = r2 * r; a.s1[1] = r2; a.s1[2] = r; a.s1[3] = 1; a.c1 = 4.0 * Ebar;
  a.src2 = prob->d2ab; a.s2[0] = r2 * r; a.s2[1] = r2; a.s2[2] = r; a.s2[3] = 1; a.c2 = 4.0 * Ebar;
  HIP_TRY(ctx, launch_permute4(GEMM_F64, a, OperandRef{D, nullptr}, s));
  HIP_TRY(ctx, launch_fill(r2 * r2, 0.0, zero, s));
  HIP_TRY(ctx, launch_vjp_fold(r, N, zero, D, Vraw, hb_raw, s));
  HIP_TRY(ctx, launch_proj(PROJ_V, r, 1.0, Vraw, V_bar, s));
  HIP_TRY(ctx, launch_proj(PROJ_SYM2, r, 1.0, hb_raw, h_bar, s));
  return ACSE_OK;
}

// ===========================================================================
// Euler iteration of Eq. (9) with the stopping rules of the method section and
// the step-size controls declared with acse_solve.  The host makes every
// decision from the FP64 scalars (E, ||R||^2) of each trial; all array work
// stays on the device.
// ===========================================================================
namespace {

struct SolveWs {
  double *g_keep, *dgamma, *dots, *part;        // r^2, r^2, 8, kDotBlocks
  double *Rbar_aa, *Rbar_ab, *Vbar, *Dbar_aa, *Dbar_ab, *hbar, *gbar;  // QUADRATIC only
};

acse_status ensure_solve_ws(acse_ctx c, bool quadratic, SolveWs &sw) {
  const int64_t r2 = (int64_t)c->r_max * c->r_max;
  const int64_t n4 = r2 * r2;
  const int64_t small = 2 * round_up(r2 * 8, 256) + round_up(8 * 8, 256) + round_up(kDotBlocks * 8, 256);
  const int64_t big = 5 * round_up(n4 * 8, 256) + 2 * round_up(r2 * 8, 256);
  const int64_t need = small + (quadratic ? big : 0);
  if (c->sbytes < need) {
    if (c->sbase) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      (void)hipFree(c->sbase);
      c->sbase = nullptr;
      c->sbytes = 0;
    }
    if (hipMalloc(&c->sbase, need) != hipSuccess) {
      (void)hipGetLastError();
      c->sbase = nullptr;
      return fail(c, ACSE_ERR_NOMEM, "driver workspace allocation failed");
    }
    c->sbytes = need;
  }
  char *p = static_cast<char *>(c->sbase);
  auto take = [&](int64_t bytes) {
    double *x = reinterpret_cast<double *>(p);
    p += round_up(bytes, 256);
    return x;
  };
  sw = SolveWs{};
  sw.g_keep = take(r2 * 8);
  sw.dgamma = take(r2 * 8);
  sw.dots = take(8 * 8);
  sw.part = take(kDotBlocks * 8);
  if (quadratic) {
    sw.Rbar_aa = take(n4 * 8);
    sw.Rbar_ab = take(n4 * 8);
    sw.Vbar = take(n4 * 8);
    sw.Dbar_aa = take(n4 * 8);
    sw.Dbar_ab = take(n4 * 8);
    sw.hbar = take(r2 * 8);
    sw.gbar = take(r2 * 8);
  }
  return ACSE_OK;
}

acse_status check_solve_options(acse_ctx c, const acse_solve_options *so, const acse_solve_result *res,
                                const acse_trial *hist, int32_t cap) {
  if (!so) return fail(c, ACSE_ERR_ARG, "solve options are NULL");
  if (!res) return fail(c, ACSE_ERR_ARG, "result is NULL");
  if (cap < 0 || (cap > 0 && !hist)) return fail(c, ACSE_ERR_ARG, "history capacity > 0 needs a history array");
  if (!std::isfinite(so->eps) || so->eps == 0.0) return fail(c, ACSE_ERR_ARG, "eps must be finite and nonzero");
  if (!std::isfinite(so->de_tol) || so->de_tol < 0.0) return fail(c, ACSE_ERR_ARG, "de_tol must be finite and >= 0");
  if (!std::isfinite(so->eps_max) || so->eps_max < 0.0) return fail(c, ACSE_ERR_ARG, "eps_max must be finite and >= 0");
  if (so->max_iter < 0) return fail(c, ACSE_ERR_ARG, "max_iter must be >= 0");
  if (so->control < ACSE_EULER_FIXED || so->control > ACSE_EULER_QUADRATIC)
    return fail(c, ACSE_ERR_ARG, "unknown step control");
  if (so->max_halvings < 0 || so->max_halvings > 60) return fail(c, ACSE_ERR_ARG, "max_halvings must be in [0, 60]");
  if (so->control == ACSE_EULER_QUADRATIC && !(so->eps > 0.0))
    return fail(c, ACSE_ERR_ARG, "the quadratic control needs eps > 0");
  if (so->reserved != 0) return fail(c, ACSE_ERR_ARG, "reserved must be 0");
  return ACSE_OK;
}

// Second step size of the quadratic control, or 0 for none: the minimiser of
// the parabola through f(0) = f0 with slope g0 and f(x) = fx, clamped to
// [x/4, min(4x, xmax)] (4x, clamped, for a non-positive curvature); none for
// g0 >= 0 or a result within 5% of x.
double quadratic_second_step(double f0, double g0, double x, double fx, double xmax) {
  if (!(g0 < 0.0)) return 0.0;
  const double c = (fx - f0 - g0 * x) / (x * x);
  const double hi = std::min(4.0 * x, xmax);
  double y = c > 0.0 ? -g0 / (2.0 * c) : hi;
  y = std::min(std::max(y, 0.25 * x), hi);
  return std::fabs(y - x) <= 0.05 * std::fabs(x) ? 0.0 : y;
}

}  // namespace

extern "C" acse_status acse_solve(acse_ctx ctx, acse_problem *prob, const acse_options *opts,
                                  const acse_solve_options *so, acse_solve_result *res,
                                  acse_trial *hist, int32_t cap) {
  acse_status st = validate(ctx, prob, opts);
  if (st != ACSE_OK) return st;
  if ((st = check_solve_options(ctx, so, res, hist, cap)) != ACSE_OK) return st;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  const bool quad = so->control == ACSE_EULER_QUADRATIC;
  if (quad && ctx->ny_on && prob->r > kSoMaxR)
    return fail(ctx, ACSE_ERR_UNSUPPORTED, "the quadratic control with NY needs the NY adjoint, which runs up to r = " +
                                               std::to_string(kSoMaxR));
  if (ctx->crt_moduli && (st = ensure_crt(ctx)) != ACSE_OK) return st;
  SolveWs sw{};
  if ((st = ensure_solve_ws(ctx, quad, sw)) != ACSE_OK) return st;
  if (quad && (st = ensure_vjp_ws(ctx)) != ACSE_OK) return st;

  Workspace &w = ctx->ws;
  hipStream_t s = ctx->stream;
  const int r = prob->r;
  const int N = prob->n_alpha + prob->n_beta;
  const int64_t r2 = (int64_t)r * r, n4 = r2 * r2;
  const GemmPrec prec = prec_of(opts);
  const int cfg = opts ? opts->tile : -1;
  bool masked = false;
  const ActiveBits act = make_bits(opts, r, &masked);
  const double eps_max = so->eps_max > 0.0 ? so->eps_max : 16.0 * std::fabs(so->eps);
  // the adjoint calls run without the input check (done once above)
  acse_options vopt{};
  if (opts) vopt = *opts;
  vopt.active = nullptr;
  vopt.flags &= ~ACSE_FLAG_CHECK_INPUTS;

  *res = acse_solve_result{};
  auto record = [&](double x, double E, double f, int n) -> int32_t {
    const int32_t id = res->trials++;
    if (id < cap) hist[id] = acse_trial{x, E, f, n, 0};
    return id;
  };
  auto mark = [&](int32_t id) { if (id >= 0 && id < cap) hist[id].accepted = 1; };
  // residual of the current problem arrays into w.Raa/Rab (masked copy into M)
  auto residual = [&](double *f, double *E) -> acse_status {
    acse_status q;
    if ((q = prep_rdm_operands(ctx, prob, prec)) != ACSE_OK) return q;
    if ((q = run_map(ctx, prob, prec, cfg, w.Aaa, w.Aab, -1.0, w.Raa, w.Rab, act, masked ? w.Maa : nullptr,
                     masked ? w.Mab : nullptr, 0)) != ACSE_OK)
      return q;
    ++res->maps;
    return fetch_scalars(ctx, f, E);
  };
  // trial 2D' = rescaled(2D_n + x U_n) from the kept 2D_n, its 1-RDM, E' and ||R'||^2
  auto trial = [&](double x, bool restore, double *f, double *E) -> acse_status {
    if (restore) {
      HIP_TRY(ctx, hipMemcpyAsync(prob->d2aa, w.Naa, n4 * 8, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(prob->d2ab, w.Nab, n4 * 8, hipMemcpyDeviceToDevice, s));
    }
    {
      StageTimer t5(ctx, 5);
      HIP_TRY(ctx, launch_step_tail(r, N, x, prob->h, prob->V, w.Uaa, w.Uab, prob->d2aa, prob->d2ab,
                                    w.scal + 4, w.partial, w.scal + 1, s));
      HIP_TRY(ctx, launch_contract_1rdm(r, N, prob->d2aa, prob->d2ab, prob->d1, s));
    }
    return residual(f, E);
  };

  {
    StageTimer t1(ctx, 1);
    HIP_TRY(ctx, launch_fold(r, N, prob->h, prob->V, w.Aaa, w.Aab, s));
  }
  {
    StageTimer t5(ctx, 5);
    HIP_TRY(ctx, launch_energy(r, N, prob->h, prob->V, prob->d2aa, prob->d2ab, w.partial, w.scal + 1, s));
  }
  double E = 0.0, f = 0.0;
  if ((st = residual(&f, &E)) != ACSE_OK) return st;
  res->energy0 = res->energy = E;
  res->norm2_0 = res->norm2 = f;
  res->stop = ACSE_STOP_MAX_ITER;
  double e = so->eps;

  for (int n = 0; n < so->max_iter; ++n) {
    // U_n = F(R_m) with the operands of 2D_n
    if ((st = run_map(ctx, prob, prec, cfg, masked ? w.Maa : w.Raa, masked ? w.Mab : w.Rab, +1.0, w.Uaa,
                      w.Uab, ActiveBits{}, nullptr, nullptr, 2)) != ACSE_OK)
      return st;
    ++res->maps;
    double g0 = 0.0;
    if (quad) {
      // f'(0) = <Dbar_aa, U_aa> + <Dbar_ab, U_ab> + <gbar, dgamma>, cotangent (4 R_aa, 8 R_ab)
      HIP_TRY(ctx, launch_scale2(n4, 4.0, w.Raa, 8.0, w.Rab, sw.Rbar_aa, sw.Rbar_ab, s));
      if ((st = acse_residual_vjp(ctx, prob, &vopt, sw.Rbar_aa, sw.Rbar_ab, sw.hbar, sw.Vbar, sw.gbar,
                                  sw.Dbar_aa, sw.Dbar_ab)) != ACSE_OK)
        return st;
      HIP_TRY(ctx, launch_contract_1rdm(r, N, w.Uaa, w.Uab, sw.dgamma, s));
      HIP_TRY(ctx, launch_dot(n4, sw.Dbar_aa, w.Uaa, sw.part, sw.dots + 0, s));
      HIP_TRY(ctx, launch_dot(n4, sw.Dbar_ab, w.Uab, sw.part, sw.dots + 1, s));
      HIP_TRY(ctx, launch_dot(r2, sw.gbar, sw.dgamma, sw.part, sw.dots + 2, s));
      double d[3] = {0.0, 0.0, 0.0};
      HIP_TRY(ctx, hipMemcpyAsync(d, sw.dots, sizeof d, hipMemcpyDeviceToHost, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
      g0 = d[0] + d[1] + d[2];
      if (!std::isfinite(g0)) return fail(ctx, ACSE_ERR_NONFINITE, "slope of ||R||^2 is not finite");
      StageTimer t1(ctx, 1);  // the adjoint reuses the fold's buffers
      HIP_TRY(ctx, launch_fold(r, N, prob->h, prob->V, w.Aaa, w.Aab, s));
    }
    // keep 2D_n and 1D_n
    HIP_TRY(ctx, hipMemcpyAsync(w.Naa, prob->d2aa, n4 * 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(w.Nab, prob->d2ab, n4 * 8, hipMemcpyDeviceToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(sw.g_keep, prob->d1, r2 * 8, hipMemcpyDeviceToDevice, s));

    auto ok = [&](double Et, double ft) { return Et <= E && ft <= f; };
    double x1 = e, f1 = 0.0, E1 = 0.0;
    if ((st = trial(x1, false, &f1, &E1)) != ACSE_OK) return st;
    int32_t id1 = record(x1, E1, f1, n);
    bool chosen = ok(E1, f1);
    double xc = x1, fc = f1, Ec = E1;  // chosen trial (valid if chosen)
    int32_t idc = id1;
    double last_E = E1;
    double cand = e;
    if (quad) {
      const double x2 = quadratic_second_step(f, g0, x1, f1, eps_max);
      if (x2 != 0.0) {
        double f2 = 0.0, E2 = 0.0;
        if ((st = trial(x2, true, &f2, &E2)) != ACSE_OK) return st;
        const int32_t id2 = record(x2, E2, f2, n);
        last_E = E2;
        const bool ok1 = ok(E1, f1), ok2 = ok(E2, f2);
        if (ok2 && (!ok1 || f2 < f1)) {
          chosen = true; xc = x2; fc = f2; Ec = E2; idc = id2;
        } else if (ok1) {
          // the arrays hold the second trial: evaluate the first again (same kernels, same values)
          if ((st = trial(x1, true, &f1, &E1)) != ACSE_OK) return st;
          chosen = true; xc = x1; fc = f1; Ec = E1; idc = id1;
        } else {
          chosen = false;
        }
        cand = std::min(x1, x2);
      }
    }
    for (int hv = 0; !chosen && so->control != ACSE_EULER_FIXED && hv < so->max_halvings; ++hv) {
      cand *= 0.5;
      double ft = 0.0, Et = 0.0;
      if ((st = trial(cand, true, &ft, &Et)) != ACSE_OK) return st;
      const int32_t id = record(cand, Et, ft, n);
      last_E = Et;
      if (ok(Et, ft)) { chosen = true; xc = cand; fc = ft; Ec = Et; idc = id; }
    }
    if (!chosen) {
      // keep the state before the rise
      HIP_TRY(ctx, hipMemcpyAsync(prob->d2aa, w.Naa, n4 * 8, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(prob->d2ab, w.Nab, n4 * 8, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipMemcpyAsync(prob->d1, sw.g_keep, r2 * 8, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
      res->stop = last_E > E ? ACSE_STOP_ENERGY_ROSE : ACSE_STOP_NORM_ROSE;
      break;
    }
    mark(idc);
    const double dE = Ec - E;
    E = Ec;
    f = fc;
    e = xc;
    res->iterations = n + 1;
    res->eps = xc;
    res->energy = E;
    res->norm2 = f;
    if (std::fabs(dE) < so->de_tol) {
      res->stop = ACSE_STOP_CONVERGED;
      break;
    }
  }
  return ACSE_OK;
}

// ===========================================================================
// Batched residual: instances of uneven r (ground and excited states, several
// molecules) share one persistent launch of all their pair-index products.
// ===========================================================================
namespace {

constexpr int kMaxBatch = 4096;
// Per-instance stages run on kBatchLanes lanes: lane 0 is the context stream,
// lanes 1.. are side streams.  With HIP's default of four hardware queues per
// process, the context stream and three side streams each get a queue of
// their own; a fourth side stream would share one and serialise two lanes.
constexpr int kBatchLanes = 4;
constexpr int kSideStreams = kBatchLanes - 1;

struct BatchPlan {
  std::vector<Workspace> ws;
  double *norms = nullptr;
  GemmProb *dprobs = nullptr;
};

std::string batch_key(GemmPrec prec, int count, const acse_problem *probs) {
  std::string k = std::to_string((int)prec) + ":";
  for (int i = 0; i < count; ++i) k += std::to_string(probs[i].r) + ",";
  return k;
}

acse_status validate_batch(acse_ctx c, int32_t count, const acse_problem *probs,
                           const acse_options *opts) {
  if (!c) return ACSE_ERR_ARG;
  if (count < 1 || count > kMaxBatch)
    return fail(c, ACSE_ERR_ARG, "count must be in [1, " + std::to_string(kMaxBatch) + "]");
  if (!probs) return fail(c, ACSE_ERR_ARG, "problems array is NULL");
  for (int i = 0; i < count; ++i) {
    acse_status st = validate(c, &probs[i], opts);
    if (st != ACSE_OK) return fail(c, st, "instance " + std::to_string(i) + ": " + c->err);
  }
  if (c->ny_on && opts->ny_sigma)
    return fail(c, ACSE_ERR_ARG, "a batch takes each instance's reference occupations from its n_alpha: "
                                 "ny_sigma must be NULL");
  if (c->crt_moduli && (c->ny_on || (opts && (opts->flags & ACSE_FLAG_BATCH_PERSISTENT))))
    return fail(c, ACSE_ERR_UNSUPPORTED, "int8 exact accumulation in a batch runs on the lanes (no "
                                         "ACSE_FLAG_BATCH_PERSISTENT) with the Valdemoro reconstruction");
  return ACSE_OK;
}

acse_status ensure_batch(acse_ctx c, int count, const acse_problem *probs, BatchPlan &plan) {
  int64_t need = 0;
  std::vector<int64_t> off(count);
  for (int i = 0; i < count; ++i) {
    Workspace tmp{};
    off[i] = need;
    need += round_up(carve(nullptr, probs[i].r, false, tmp), 256);
  }
  const int64_t norms_off = need;
  need += round_up((int64_t)count * 8, 256);
  const int64_t probs_off = need;
  need += round_up((int64_t)count * kProbsPerMap * (int64_t)sizeof(GemmProb), 256);
  if (need > c->bbytes) {
    if (c->bbase) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      (void)hipFree(c->bbase);
      c->bbase = nullptr;
      c->bbytes = 0;
    }
    if (hipMalloc(&c->bbase, need) != hipSuccess) {
      (void)hipGetLastError();
      c->bbase = nullptr;
      return fail(c, ACSE_ERR_NOMEM, "batch workspace allocation failed");
    }
    c->bbytes = need;
    HIP_TRY(c, launch_fill(need / 8, 0.0, static_cast<double *>(c->bbase), c->stream));
  }
  if (kProbsPerMap * count > c->hdesc_cap) {
    if (c->hdesc) {
      if (c->hdesc_done) HIP_TRY(c, hipEventSynchronize(c->hdesc_done));
      (void)hipHostFree(c->hdesc);
      c->hdesc = nullptr;
      c->hdesc_cap = 0;
    }
    HIP_TRY(c, hipHostMalloc(reinterpret_cast<void **>(&c->hdesc), kProbsPerMap * count * sizeof(GemmProb),
                             hipHostMallocDefault));
    c->hdesc_cap = kProbsPerMap * count;
  }
  if (!c->hdesc_done) HIP_TRY(c, hipEventCreateWithFlags(&c->hdesc_done, hipEventDisableTiming));
  if (!c->fork_ev) HIP_TRY(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
  for (int q = 0; q < kSideStreams; ++q) {
    if (!c->side[q]) HIP_TRY(c, hipStreamCreateWithFlags(&c->side[q], hipStreamNonBlocking));
    if (!c->join_ev[q]) HIP_TRY(c, hipEventCreateWithFlags(&c->join_ev[q], hipEventDisableTiming));
  }
  char *base = static_cast<char *>(c->bbase);
  plan.ws.assign(count, Workspace{});
  for (int i = 0; i < count; ++i) carve(base + off[i], probs[i].r, false, plan.ws[i]);
  plan.norms = reinterpret_cast<double *>(base + norms_off);
  plan.dprobs = reinterpret_cast<GemmProb *>(base + probs_off);
  return ACSE_OK;
}

int batch_cfg_default(GemmPrec prec, int count, const acse_problem *probs) {
  int64_t rmax = 0;
  for (int i = 0; i < count; ++i) rmax = std::max<int64_t>(rmax, probs[i].r);
  return gemm_default_cfg(prec, (int)(rmax * rmax), (int)(rmax * rmax));
}

int batch_cfg(acse_ctx c, GemmPrec prec, int count, const acse_problem *probs, int tile) {
  if (tile >= 0) return tile;
  auto it = c->tuned_batch.find(batch_key(prec, count, probs));
  if (it != c->tuned_batch.end()) return it->second;
  return batch_cfg_default(prec, count, probs);
}

// Routes the library's launches to another stream for a scope.
struct StreamSwap {
  acse_ctx c;
  hipStream_t saved;
  StreamSwap(acse_ctx c_, hipStream_t to) : c(c_), saved(c_->stream) { c->stream = to; }
  ~StreamSwap() { c->stream = saved; }
};

// Stream of lane l (lane 0: the context stream).
hipStream_t lane_stream(acse_ctx c, int l) { return l == 0 ? c->stream : c->side[l - 1]; }

// The side streams of lanes 1 .. ns-1 wait for everything enqueued so far on
// the context stream (lane 0).
acse_status fork_sides(acse_ctx c, int ns) {
  HIP_TRY(c, hipEventRecord(c->fork_ev, c->stream));
  for (int q = 0; q + 1 < ns; ++q) HIP_TRY(c, hipStreamWaitEvent(c->side[q], c->fork_ev, 0));
  return ACSE_OK;
}
// The context stream waits for everything enqueued so far on those side streams.
acse_status join_sides(acse_ctx c, int ns) {
  for (int q = 0; q + 1 < ns; ++q) {
    HIP_TRY(c, hipEventRecord(c->join_ev[q], c->side[q]));
    HIP_TRY(c, hipStreamWaitEvent(c->stream, c->join_ev[q], 0));
  }
  return ACSE_OK;
}

// Tile configuration of one instance's products: the caller's, else the one
// tuned for (r, precision), else the size default (as a single call takes it).
int instance_cfg(acse_ctx c, GemmPrec prec, int r, int tile) {
  if (tile >= 0) return tile;
  auto it = c->tuned.find({r, (int)prec});
  return it != c->tuned.end() ? it->second : gemm_default_cfg(prec, r * r, r * r);
}

// Lanes: every instance runs its whole residual (RDM operands, fold,
// transforms, its own grouped product launch, assembly) in order on one side
// stream, so the memory-bound stages of one instance overlap the products of
// another.  Each instance's launches are those of a single acse_residual call
// with the same tile configuration.
acse_status run_lanes(acse_ctx c, int count, const acse_problem *probs, GemmPrec prec, int tile,
                      double *const *Raa, double *const *Rab, BatchPlan &plan, const std::vector<int> &order,
                      const std::vector<int> &lane, int ns) {
  acse_status st;
  if (prec == GEMM_I8CRT) {
    // one residue workspace per lane: the instances of a lane run in order
    for (int q = 0; q < ns; ++q)
      if ((st = alloc_crt_ws(c, c->lane_cw[q])) != ACSE_OK) return st;
    for (int i = 0; i < count; ++i) plan.ws[i].crt = &c->lane_cw[lane[i]];
  }
  if ((st = fork_sides(c, ns)) != ACSE_OK) return st;
  const ActiveBits none{};
  auto one = [&](int i) -> acse_status {
    const acse_problem *p = &probs[i];
    Workspace &w = plan.ws[i];
    StreamSwap sw(c, lane_stream(c, lane[i]));
    acse_status s2 = prep_rdm_operands(c, p, prec, w);
    if (s2 != ACSE_OK) return s2;
    {
      StageTimer t1(c, 1);
      HIP_TRY(c, launch_fold(p->r, p->n_alpha + p->n_beta, p->h, p->V, w.Aaa, w.Aab, c->stream));
    }
    if ((s2 = map_front(c, p, prec, w.Aaa, w.Aab, w)) != ACSE_OK) return s2;
    GemmBatch b{};
    b.count = kProbsPerMap;
    if (prec == GEMM_I8CRT) {
      map_probs_crt(c, w, p->r, b.p);
      {
        StageTimer t3(c, 3);
        HIP_TRY(c, gemm_crt_launch(b, c->crt, c->stream));
      }
      StageTimer t4(c, 4);
      HIP_TRY(c, crt_combine_launch(b, c->crt, c->stream));
    } else {
      map_probs(w, prec, p->r, b.p);
      StageTimer t3(c, 3);
      HIP_TRY(c, gemm_launch(prec, instance_cfg(c, prec, p->r, tile), b, c->stream));
    }
    return map_back(c, p, -1.0, Raa ? Raa[i] : w.Raa, Rab ? Rab[i] : w.Rab, none, nullptr, nullptr,
                    plan.norms + i, w);
  };
  // each lane's instances in decreasing size; with the int8, FP32 and split-BF16
  // products every second lane takes its own in increasing size, so that the
  // lanes' memory-bound fronts and compute-bound products fall at different
  // times (the FP64 products, which dominate each instance more, keep the
  // decreasing order there); issued round-robin over the lanes so that every
  // lane starts at once
  std::vector<std::vector<int>> per(ns);
  for (int i : order) per[lane[i]].push_back(i);
  if (prec != GEMM_F64)
    for (int q = 1; q < ns; q += 2) std::reverse(per[q].begin(), per[q].end());
  size_t depth = 0;
  for (int q = 0; q < ns; ++q) depth = std::max(depth, per[q].size());
  st = ACSE_OK;
  for (size_t t = 0; t < depth && st == ACSE_OK; ++t)
    for (int q = 0; q < ns && st == ACSE_OK; ++q)
      if (t < per[q].size()) st = one(per[q][t]);
  // a failing launch still rejoins the side streams before returning
  const acse_status sj = join_sides(c, ns);
  return st != ACSE_OK ? st : sj;
}

// Per-instance stages run concurrently on the side streams (largest instances
// first, each to the least loaded stream).  Default: lanes (above).  With
// `persistent` (and always with the NY 3-RDM) the products of all instances
// run as one persistent launch on the context stream between the fronts and
// the back ends.
acse_status run_batched(acse_ctx c, int count, const acse_problem *probs, GemmPrec prec, int cfg,
                        double *const *Raa, double *const *Rab, BatchPlan &plan, bool persistent, int tile) {
  acse_status st;
  const int ns = std::min(count, kBatchLanes);
  std::vector<int> order(count), lane(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return probs[a].r > probs[b].r; });
  double load[kBatchLanes] = {};
  for (int i : order) {
    int best = 0;
    for (int q = 1; q < ns; ++q)
      if (load[q] < load[best]) best = q;
    lane[i] = best;
    const double rr = probs[i].r;
    load[best] += rr * rr * rr * rr * rr;
  }
  if (!persistent && !c->ny_on) return run_lanes(c, count, probs, prec, tile, Raa, Rab, plan, order, lane, ns);
  std::vector<GemmProb> gp(kProbsPerMap * (size_t)count);
  if ((st = fork_sides(c, ns)) != ACSE_OK) return st;
  // a failing launch still rejoins the side streams before returning
  auto front = [&](int i) -> acse_status {
    const acse_problem *p = &probs[i];
    Workspace &w = plan.ws[i];
    StreamSwap sw(c, lane_stream(c, lane[i]));
    acse_status s2 = prep_rdm_operands(c, p, prec, w);
    if (s2 != ACSE_OK) return s2;
    {
      StageTimer t1(c, 1);
      HIP_TRY(c, launch_fold(p->r, p->n_alpha + p->n_beta, p->h, p->V, w.Aaa, w.Aab, c->stream));
    }
    if ((s2 = map_front(c, p, prec, w.Aaa, w.Aab, w)) != ACSE_OK) return s2;
    map_probs(w, prec, p->r, &gp[kProbsPerMap * (size_t)i]);
    return ACSE_OK;
  };
  for (int i : order)
    if ((st = front(i)) != ACSE_OK) {
      (void)join_sides(c, ns);
      return st;
    }
  if ((st = join_sides(c, ns)) != ACSE_OK) return st;
  {
    // the pinned staging buffer may still feed the previous call's copy
    HIP_TRY(c, hipEventSynchronize(c->hdesc_done));
    StageTimer t3(c, 3);
    HIP_TRY(c, gemm_launch_persistent(prec, cfg, gp, c->hdesc, plan.dprobs, c->stream));
    HIP_TRY(c, hipEventRecord(c->hdesc_done, c->stream));
  }
  const ActiveBits none{};
  if (c->ny_on) {
    // the NY share uses one workspace per context: the back ends run in order
    // on the context's stream, each with its instance's reference occupations
    for (int i : order) {
      const acse_problem *p = &probs[i];
      c->ny_sigma.assign(p->r, -1.0);
      for (int q = 0; q < p->n_alpha; ++q) c->ny_sigma[q] = 1.0;
      if ((st = map_back(c, p, -1.0, Raa ? Raa[i] : plan.ws[i].Raa, Rab ? Rab[i] : plan.ws[i].Rab, none,
                         nullptr, nullptr, plan.norms + i, plan.ws[i], plan.ws[i].Aaa, plan.ws[i].Aab,
                         prec, cfg)) != ACSE_OK)
        return st;
    }
    return ACSE_OK;
  }
  if ((st = fork_sides(c, ns)) != ACSE_OK) return st;
  for (int i : order) {
    StreamSwap sw(c, lane_stream(c, lane[i]));
    if ((st = map_back(c, &probs[i], -1.0, Raa ? Raa[i] : plan.ws[i].Raa,
                       Rab ? Rab[i] : plan.ws[i].Rab, none, nullptr, nullptr, plan.norms + i,
                       plan.ws[i])) != ACSE_OK)
      break;
  }
  const acse_status sj = join_sides(c, ns);
  return st != ACSE_OK ? st : sj;
}

}  // namespace

extern "C" acse_status acse_residual_batched(acse_ctx ctx, int32_t count, const acse_problem *probs,
                                             const acse_options *opts, double *const *R_aa,
                                             double *const *R_ab, double *norm2_host) {
  acse_status st = validate_batch(ctx, count, probs, opts);
  if (st != ACSE_OK) return st;
  if (!R_aa || !R_ab) return fail(ctx, ACSE_ERR_ARG, "output pointer arrays are NULL");
  for (int i = 0; i < count; ++i) {
    if ((st = check_out(ctx, R_aa[i], "R_aa[i]")) != ACSE_OK) return st;
    if ((st = check_out(ctx, R_ab[i], "R_ab[i]")) != ACSE_OK) return st;
  }
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (ctx->crt_moduli && (st = ensure_crt(ctx)) != ACSE_OK) return st;
  const GemmPrec prec = prec_of(opts);
  BatchPlan plan;
  if ((st = ensure_batch(ctx, count, probs, plan)) != ACSE_OK) return st;
  const int tile = opts ? opts->tile : -1;
  const bool persistent = opts && (opts->flags & ACSE_FLAG_BATCH_PERSISTENT);
  const int cfg = batch_cfg(ctx, prec, count, probs, tile);
  if ((st = run_batched(ctx, count, probs, prec, cfg, R_aa, R_ab, plan, persistent, tile)) != ACSE_OK) return st;
  if (norm2_host) {
    HIP_TRY(ctx, hipMemcpyAsync(norm2_host, plan.norms, count * sizeof(double), hipMemcpyDeviceToHost,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < count; ++i)
      if (!std::isfinite(norm2_host[i]))
        return fail(ctx, ACSE_ERR_NONFINITE, "||R||^2 of instance " + std::to_string(i) + " is not finite");
  }
  return ACSE_OK;
}

extern "C" acse_status acse_autotune_batched(acse_ctx ctx, int32_t count, const acse_problem *probs,
                                             const acse_options *opts, int32_t *best_tile,
                                             double *times_ms) {
  acse_status st = validate_batch(ctx, count, probs, opts);
  if (st != ACSE_OK) return st;
  ctx->ny_on = false;  // the tile choice concerns the Valdemoro products
  if (!best_tile) return fail(ctx, ACSE_ERR_ARG, "best_tile is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  if (!(opts && (opts->flags & ACSE_FLAG_BATCH_PERSISTENT))) {
    // lanes: each instance's products are a single call's, so tune each r as
    // acse_autotune does (cached per (r, precision)); report the largest r
    int big = 0;
    for (int i = 1; i < count; ++i)
      if (probs[i].r > probs[big].r) big = i;
    std::vector<int> seen;
    for (int i = 0; i < count; ++i) {
      if (std::find(seen.begin(), seen.end(), probs[i].r) != seen.end()) continue;
      seen.push_back(probs[i].r);
      int32_t b = -1;
      double t[ACSE_NUM_TILE_CONFIGS] = {};
      if ((st = acse_autotune(ctx, &probs[i], opts, &b, t)) != ACSE_OK)
        return fail(ctx, st, "instance " + std::to_string(i) + ": " + ctx->err);
      if (probs[i].r == probs[big].r) {
        *best_tile = b;
        if (times_ms)
          for (int q = 0; q < ACSE_NUM_TILE_CONFIGS; ++q) times_ms[q] = t[q];
      }
    }
    return ACSE_OK;
  }
  const GemmPrec prec = prec_of(opts);
  BatchPlan plan;
  if ((st = ensure_batch(ctx, count, probs, plan)) != ACSE_OK) return st;
  const bool was = ctx->profiling;
  auto saved = std::move(ctx->recs);
  ctx->recs.clear();
  double best = 1e300;
  int arg = 0;
  double tms[ACSE_NUM_TILE_CONFIGS] = {};
  for (int cfg = 0; cfg < ACSE_NUM_TILE_CONFIGS; ++cfg) {
    ctx->profiling = false;
    if ((st = run_batched(ctx, count, probs, prec, cfg, nullptr, nullptr, plan, true, cfg)) != ACSE_OK) break;
    ctx->profiling = true;
    for (int rep = 0; rep < kTuneReps && st == ACSE_OK; ++rep)
      st = run_batched(ctx, count, probs, prec, cfg, nullptr, nullptr, plan, true, cfg);
    if (st != ACSE_OK) break;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) { st = fail(ctx, ACSE_ERR_HIP, "sync"); break; }
    double ms = 1e300;  // fastest of the timed repetitions (robust to interference)
    for (auto &q : ctx->recs) {
      if (q.stage == 3) {
        float e = 0.0f;
        (void)hipEventElapsedTime(&e, q.a, q.b);
        ms = std::min(ms, (double)e);
      }
      ctx->pool.push_back(q.a);
      ctx->pool.push_back(q.b);
    }
    ctx->recs.clear();
    tms[cfg] = ms;
    if (times_ms) times_ms[cfg] = ms;
    if (ms < best) { best = ms; arg = cfg; }
  }
  ctx->profiling = was;
  ctx->recs = std::move(saved);
  if (st != ACSE_OK) return st;
  arg = keep_default(arg, best, batch_cfg_default(prec, count, probs), tms);
  ctx->tuned_batch[batch_key(prec, count, probs)] = arg;
  *best_tile = arg;
  return ACSE_OK;
}

// ===========================================================================
// States of any S_z (N_alpha != N_beta): the three unique spin blocks
// (alpha-alpha, beta-beta, alpha-beta) and one 1-RDM per spin.
//
// The map F(X) runs over spin-orbital tensors held as spatial spin blocks
// (block b: bit 3 - t set when index t is beta).  With X_A the
// pair-antisymmetrised X, W = Gamma2 - 2/3 Gamma1^Gamma1 and Gamma1 =
// diag(ga, gb):
//   Y^{ij}_{kl} = sum_rs Gamma2^{ij}_{rs} X_A^{kl}_{rs}
//   H^{kl}_{rs} = sum_p X_A^{kp}_{rs} Gamma1_pl,   f_ks = sum_r H^{kr}_{rs}
//   t_jk = sum_prs W^{jp}_{rs} X_A^{kp}_{rs},      Xt^{kp}_{is} = sum_r Gamma1_ir X_A^{kp}_{rs}
//   E^{ij}_{kl} = 2 sum_ps Xt^{kp}_{is} W^{jp}_{sl}
//   T = sum_rs W^{ij}_{rs} H^{kl}_{rs} + 2 sum_s f_ks W^{ij}_{sl} + Gamma1_il t_jk
//       - Gamma1_jl t_ik + E^{ij}_{kl} - E^{ji}_{kl}
//   S = Y - (T - T(k<->l)),   F = S - S^T (Hermitian X) or S + S^T (anti-Hermitian X)
// (the Valdemoro 3-RDM of App. C folded in as in the singlet path).  Only the
// blocks that reach F's alpha-alpha, beta-beta and alpha-beta outputs are
// formed; a summed pair antisymmetric in both operands with opposite spins is
// taken once with weight 2.  17 r^2 x r^2 x r^2 FP64 products per map (Y 3,
// the W H products 4, E 10), grouped in three launches.
// ===========================================================================

namespace {

constexpr int kSpinNat = 50;   // natural r^4 arrays
constexpr int kSpinOps = 25;   // GEMM operand buffers
enum { B0000 = 0, B0101 = 5, B0110 = 6, B1001 = 9, B1010 = 10, B1111 = 15 };
constexpr int kSix[6] = {B0000, B1111, B0101, B1010, B0110, B1001};
inline int spin_of(int b, int t) { return (b >> (3 - t)) & 1; }

struct SpinWs {
  double *XA[16] = {}, *H[16] = {}, *Xt[16] = {}, *W[16] = {}, *Y[16] = {}, *T[16] = {}, *E[16] = {}, *S[16] = {};
  double *R[3] = {}, *U[3] = {}, *Rm[3] = {};
  double *G2p[16] = {}, *Wp[16] = {}, *WPp[16] = {}, *XAp[16] = {}, *Hp[16] = {}, *XtP[16] = {};
  double *f[2] = {}, *t[2] = {}, *part = nullptr, *scal = nullptr;
  double *ops[kSpinOps] = {};  // every GEMM operand buffer, in allocation order
  // results of the four pair-packed products (rows i < j), row-major [pairs][r^2]
  double *Pk[4] = {};
  // int8 exact-accumulation products (allocated by the first such call): the
  // residue planes and row exponents of each operand buffer, and the residues
  // of one launch's products
  void *cbase = nullptr;
  int8_t *cres[kSpinOps] = {};
  int *cexp[kSpinOps] = {};
  int8_t *cy = nullptr;
  // the state 2D_n, 1D_n kept while the Euler driver runs its trials
  // (allocated by the first acse_solve_spin call)
  void *kbase = nullptr;
  double *Nk[3] = {}, *gk[2] = {};
  // the quadratic control's slope (allocated by its first use): R_n kept, the
  // five-point combination of the residuals along the line, the 1-RDMs of U
  void *qbase = nullptr;
  double *Rk[3] = {}, *Qa[3] = {}, *dg[2] = {};
};

acse_status ensure_spin_ws(acse_ctx c, SpinWs *&out) {
  if (c->spws) { out = static_cast<SpinWs *>(c->spws); return ACSE_OK; }
  const int rm = c->r_max;
  const int64_t r2 = (int64_t)rm * rm;
  const int64_t nat = round_up(r2 * r2 * 8, 256);
  const int64_t opb = round_up(op_rows(rm) * op_ld(rm) * 8, 256);
  const int64_t small = round_up((4 * r2 + (int64_t)t_partial_blocks() * r2 + kDotBlocks + 64) * 8, 256);
  const int64_t bytes = kSpinNat * nat + kSpinOps * opb + small;
  if (hipMalloc(&c->spbase, bytes) != hipSuccess) {
    (void)hipGetLastError();
    c->spbase = nullptr;
    return fail(c, ACSE_ERR_NOMEM, "cannot allocate the spin-block workspace (" + std::to_string(bytes) + " bytes)");
  }
  c->spbytes = bytes;
  // operand padding rows are read by full tiles: give every byte a defined value once
  if (launch_fill((kSpinOps * opb) / 8, 0.0, reinterpret_cast<double *>(static_cast<char *>(c->spbase) + kSpinNat * nat),
                  c->stream) != hipSuccess)
    return fail(c, ACSE_ERR_HIP, "spin workspace fill failed");
  SpinWs w;
  char *q = static_cast<char *>(c->spbase);
  auto take_nat = [&]() { double *x = reinterpret_cast<double *>(q); q += nat; return x; };
  for (int b : kSix) { w.XA[b] = take_nat(); w.Xt[b] = take_nat(); w.W[b] = take_nat(); w.E[b] = take_nat(); }
  for (int b : {B0000, B1111, B0101, B1001, B0110}) w.H[b] = take_nat();
  for (int b : {B0000, B1111, B0101}) { w.Y[b] = take_nat(); w.S[b] = take_nat(); }
  for (int b : {B0000, B1111, B0101, B0110}) w.T[b] = take_nat();
  for (int k = 0; k < 3; ++k) { w.R[k] = take_nat(); w.U[k] = take_nat(); w.Rm[k] = take_nat(); }
  {  // two packed results (r(r-1)/2 x r^2 doubles each) per natural array
    double *a = take_nat(), *b = take_nat();
    const int64_t half = (int64_t)npair_lt(rm) * rm * rm;
    w.Pk[0] = a; w.Pk[1] = a + half; w.Pk[2] = b; w.Pk[3] = b + half;
  }
  int nops = 0;
  auto take_op = [&]() {
    double *x = reinterpret_cast<double *>(q);
    q += opb;
    w.ops[nops++] = x;
    return x;
  };
  for (int b : {B0000, B1111, B0101}) { w.G2p[b] = take_op(); w.Wp[b] = take_op(); w.XAp[b] = take_op(); }
  for (int b : kSix) { w.WPp[b] = take_op(); w.XtP[b] = take_op(); }
  for (int b : {B0000, B1111, B0101, B1001}) w.Hp[b] = take_op();
  double *sm = reinterpret_cast<double *>(q);
  w.f[0] = sm; w.f[1] = sm + r2; w.t[0] = sm + 2 * r2; w.t[1] = sm + 3 * r2;
  w.part = sm + 4 * r2;
  w.scal = w.part + (int64_t)t_partial_blocks() * r2 + kDotBlocks;
  SpinWs *keep = new (std::nothrow) SpinWs(w);
  if (!keep) return fail(c, ACSE_ERR_NOMEM, "cannot allocate the spin workspace table");
  c->spws = keep;
  out = keep;
  return ACSE_OK;
}

acse_status validate_spin(acse_ctx c, const acse_problem_spin *p, const acse_options *o, bool need_d1) {
  if (!c) return ACSE_ERR_ARG;
  if (!p) return fail(c, ACSE_ERR_ARG, "problem is NULL");
  if (p->r < 2 || p->r > c->r_max)
    return fail(c, ACSE_ERR_SHAPE, "r = " + std::to_string(p->r) + " outside [2, r_max = " +
                                       std::to_string(c->r_max) + "]");
  const int N = p->n_alpha + p->n_beta;
  if (p->n_alpha < 0 || p->n_beta < 0 || N < 2 || p->n_alpha > p->r || p->n_beta > p->r)
    return fail(c, ACSE_ERR_SHAPE, "electron counts must satisfy N >= 2 and n_sigma <= r");
  const void *ptrs[7] = {p->h, p->V, p->d2aa, p->d2bb, p->d2ab, p->d1a, p->d1b};
  for (int k = 0; k < (need_d1 ? 7 : 5); ++k) {
    if (!ptrs[k]) return fail(c, ACSE_ERR_ARG, "a problem pointer is NULL");
    if (!aligned16(ptrs[k])) return fail(c, ACSE_ERR_ALIGN, "problem arrays must be 16-byte aligned");
  }
  if (o) {
    if (o->precision < ACSE_FP64 || o->precision > ACSE_INT8CRT)
      return fail(c, ACSE_ERR_ARG, "unknown precision");
    if (o->precision != ACSE_FP64 && o->precision != ACSE_INT8CRT)
      return fail(c, ACSE_ERR_UNSUPPORTED, "the spin-block path runs its products in FP64 or int8 exact "
                                           "accumulation only");
    if (o->moduli != 0 && (o->moduli < kMinModuli || o->moduli > kMaxModuli))
      return fail(c, ACSE_ERR_ARG, "moduli must be 0 or in [" + std::to_string(kMinModuli) + ", " +
                                       std::to_string(kMaxModuli) + "]");
    if (o->reconstruction != ACSE_RECON_V && o->reconstruction != ACSE_RECON_NY)
      return fail(c, ACSE_ERR_ARG, "unknown reconstruction");
    if (o->reconstruction == ACSE_RECON_NY) {
      if (p->r > kSoMaxR)
        return fail(c, ACSE_ERR_UNSUPPORTED, "the NY share of the spin-block path runs up to r = " +
                                                 std::to_string(kSoMaxR));
      if (o->ny_sigma)
        for (int q = 0; q < 2 * p->r; ++q)
          if (o->ny_sigma[q] != 1 && o->ny_sigma[q] != -1)
            return fail(c, ACSE_ERR_ARG, "ny_sigma entries must be +1 or -1");
    }
    if (o->flags & ~ACSE_FLAG_GENERAL_KERNELS)
      return fail(c, (o->flags & ~(ACSE_FLAG_GENERAL_KERNELS | ACSE_FLAG_CHECK_INPUTS |
                                   ACSE_FLAG_BATCH_PERSISTENT)) ? ACSE_ERR_ARG
                                                                                         : ACSE_ERR_UNSUPPORTED,
                  "the spin-block path accepts ACSE_FLAG_GENERAL_KERNELS only");
    if (o->tile < -1 || o->tile >= gemm_num_tiles(GEMM_F64)) return fail(c, ACSE_ERR_ARG, "tile configuration out of range");
  }
  c->general = o && (o->flags & ACSE_FLAG_GENERAL_KERNELS);
  c->crt_moduli = (o && o->precision == ACSE_INT8CRT) ? (o->moduli ? o->moduli : kDefaultModuli) : 0;
  // spin-orbital reference occupations, alpha orbitals first
  c->ny_on = o && o->reconstruction == ACSE_RECON_NY;
  if (c->ny_on) {
    const int r = p->r;
    c->ny_sigma.assign(2 * r, -1.0);
    for (int q = 0; q < 2 * r; ++q)
      c->ny_sigma[q] = o->ny_sigma ? (double)o->ny_sigma[q] : (q % r < (q < r ? p->n_alpha : p->n_beta) ? 1.0 : -1.0);
  }
  return ACSE_OK;
}

// Residue workspace of the spin-block products (first int8 call) and the
// moduli table of the call in progress.
acse_status ensure_spin_crt(acse_ctx c, SpinWs &w) {
  if (!w.cbase) {
    const int rm = c->r_max;
    const int64_t r2 = (int64_t)rm * rm;
    const int64_t rbytes = round_up((int64_t)kMaxModuli * op_rows(rm) * crt_ldr((int)r2), 256);
    const int64_t ebytes = round_up(op_rows(rm) * (int64_t)sizeof(int), 256);
    const int64_t ybytes = round_up(6 * (int64_t)kMaxModuli * crt_residue_out_bytes((int)r2, (int)r2), 256);
    const int64_t bytes = kSpinOps * (rbytes + ebytes) + ybytes;
    if (hipMalloc(&w.cbase, bytes) != hipSuccess) {
      (void)hipGetLastError();
      w.cbase = nullptr;
      return fail(c, ACSE_ERR_NOMEM, "cannot allocate the int8 residue workspace of the spin-block path (" +
                                         std::to_string(bytes) + " bytes)");
    }
    char *q = static_cast<char *>(w.cbase);
    for (int k = 0; k < kSpinOps; ++k) {
      w.cres[k] = reinterpret_cast<int8_t *>(q);
      q += rbytes;
      w.cexp[k] = reinterpret_cast<int *>(q);
      q += ebytes;
    }
    w.cy = reinterpret_cast<int8_t *>(q);
  }
  if (c->crt.nmod != c->crt_moduli && !crt_table(c->crt_moduli, c->crt))
    return fail(c, ACSE_ERR_ARG, "no moduli table for " + std::to_string(c->crt_moduli) + " moduli");
  return ACSE_OK;
}

int spin_op_index(const SpinWs &w, const double *op) {
  for (int k = 0; k < kSpinOps; ++k)
    if (w.ops[k] == op) return k;
  return -1;
}

// Layout of an operand buffer: the same-spin Y and W H products run with
// their summed pair (r, s) packed to r < s (K = r(r-1)/2, row stride
// ld_pair_lt) and their A rows to the pairs i < j; every other operand has
// r^2 rows over K = r^2.
struct SpinOpShape {
  int rows, K;
  int64_t ld;
};
SpinOpShape spin_op_shape(const SpinWs &w, const double *op, int r) {
  const int r2 = r * r, nlt = npair_lt(r);
  for (int b : {B0000, B1111}) {
    if (op == w.G2p[b] || op == w.Wp[b]) return {nlt, nlt, ld_pair_lt(r)};
    if (op == w.XAp[b] || op == w.Hp[b]) return {r2, nlt, ld_pair_lt(r)};
  }
  return {r2, r2, op_ld(r)};
}

// FP64 spin operands (layouts of spin_op_shape) -> residue planes and row
// exponents; premul for the operands built from the 2-RDM (one per product).
acse_status spin_residues(acse_ctx c, SpinWs &w, int r, const std::vector<const double *> &ops, bool premul) {
  for (size_t first = 0; first < ops.size(); first += kMaxResidueJobs) {
    ResidueBatch b{};
    int rows = 0;
    for (size_t q = first; q < ops.size() && b.count < kMaxResidueJobs; ++q) {
      const int k = spin_op_index(w, ops[q]);
      if (k < 0) return fail(c, ACSE_ERR_HIP, "internal: unknown spin operand buffer");
      const SpinOpShape sh = spin_op_shape(w, ops[q], r);
      ResidueJob &J = b.job[b.count++];
      J.src = ops[q];
      J.dst = w.cres[k];
      J.e = w.cexp[k];
      J.plane = op_rows(r) * crt_ldr(sh.K);
      J.row_begin = rows;
      J.K = sh.K;
      J.ld = (int)sh.ld;
      J.ldr = (int)crt_ldr(sh.K);
      J.kbits = crt_kbits(c->crt, sh.K);
      J.premul = premul ? 1 : 0;
      rows += sh.rows;
    }
    b.total_rows = rows;
    HIP_TRY(c, launch_to_residues(b, c->crt, c->stream));
  }
  return ACSE_OK;
}

// Pair-packed operand from a natural block antisymmetric in its last pair (r,s):
// rows the pairs i < j (rows_mode 1) or all (k,l) (rows_mode 0), K the pairs
// r < s, row stride ld_pair_lt, K padding zero.
hipError_t launch_spin_pack_lt(int r, const double *in, double coef, int rows_mode, double *out, hipStream_t s) {
  PairPackArgs a{};
  const int64_t r2 = (int64_t)r * r;
  a.r = r;
  a.rows_mode = rows_mode;
  a.k_le = 0;
  a.ld = ld_pair_lt(r);
  a.nterms = 1;
  a.src[0] = in;
  a.st[0][0] = r2 * r; a.st[0][1] = r2; a.st[0][2] = r; a.st[0][3] = 1;
  a.c[0] = coef;
  a.offdiag[0] = 0;
  return launch_pack_pairs(GEMM_F64, a, OperandRef{out, nullptr}, s);
}

// W (natural, six blocks) and the RDM-side GEMM operands of a step.
acse_status spin_prep(acse_ctx c, SpinWs &w, const acse_problem_spin *p) {
  const int r = p->r;
  const int ld = (int)op_ld(r);
  hipStream_t s = c->stream;
  StageTimer timer(c, 0);
  const double *ga = p->d1a, *gb = p->d1b;
  auto comb1 = [&](double *out, const double *in, double coef, int f0, int f1, int f2, int f3) {
    Terms4 T{};
    T.n = 1;
    T.t[0] = term4(in, coef, r, f0, f1, f2, f3);
    return launch_combine4(r, T, out, 0, nullptr, s);
  };
  const double c23 = 2.0 / 3.0;
  // W = Gamma2 - 2/3 (g_pr g_qs - g_ps g_qr) per block
  HIP_TRY(c, comb1(w.W[B0000], p->d2aa, 2.0, 0, 1, 2, 3));
  HIP_TRY(c, launch_outer4(r, -c23, ga, 0, 2, ga, 1, 3, w.W[B0000], s));
  HIP_TRY(c, launch_outer4(r, c23, ga, 0, 3, ga, 1, 2, w.W[B0000], s));
  HIP_TRY(c, comb1(w.W[B1111], p->d2bb, 2.0, 0, 1, 2, 3));
  HIP_TRY(c, launch_outer4(r, -c23, gb, 0, 2, gb, 1, 3, w.W[B1111], s));
  HIP_TRY(c, launch_outer4(r, c23, gb, 0, 3, gb, 1, 2, w.W[B1111], s));
  HIP_TRY(c, comb1(w.W[B0101], p->d2ab, 2.0, 0, 1, 2, 3));                 // 2D(pa qb|ra sb)
  HIP_TRY(c, launch_outer4(r, -c23, ga, 0, 2, gb, 1, 3, w.W[B0101], s));
  HIP_TRY(c, comb1(w.W[B1010], p->d2ab, 2.0, 1, 0, 3, 2));                 // 2D(pb qa|rb sa) = d2ab[q,p,s,r]
  HIP_TRY(c, launch_outer4(r, -c23, gb, 0, 2, ga, 1, 3, w.W[B1010], s));
  HIP_TRY(c, comb1(w.W[B0110], p->d2ab, -2.0, 0, 1, 3, 2));                // 2D(pa qb|rb sa) = -d2ab[p,q,s,r]
  HIP_TRY(c, launch_outer4(r, c23, ga, 0, 3, gb, 1, 2, w.W[B0110], s));
  HIP_TRY(c, comb1(w.W[B1001], p->d2ab, -2.0, 1, 0, 2, 3));                // 2D(pb qa|ra sb) = -d2ab[q,p,r,s]
  HIP_TRY(c, launch_outer4(r, c23, gb, 0, 3, ga, 1, 2, w.W[B1001], s));
  // operands: Gamma2 and W blocks as [(ij)][(rs)], W blocks as [(jl)][(ps)] from W[j,p,s,l]
  auto pack1 = [&](double *out, const double *in, double coef, int f0, int f1, int f2, int f3) {
    Terms4 T{};
    T.n = 1;
    T.t[0] = term4(in, coef, r, f0, f1, f2, f3);
    return launch_pack_op4(r, T, out, ld, s);
  };
  // same-spin Gamma2 and W: rows i < j, K r < s
  auto packlt = [&](double *out, const double *in, double coef) {
    return launch_spin_pack_lt(r, in, coef, 1, out, s);
  };
  HIP_TRY(c, packlt(w.G2p[B0000], p->d2aa, 2.0));
  HIP_TRY(c, packlt(w.G2p[B1111], p->d2bb, 2.0));
  HIP_TRY(c, pack1(w.G2p[B0101], p->d2ab, 2.0, 0, 1, 2, 3));
  for (int b : {B0000, B1111}) HIP_TRY(c, packlt(w.Wp[b], w.W[b], 1.0));
  HIP_TRY(c, pack1(w.Wp[B0101], w.W[B0101], 1.0, 0, 1, 2, 3));
  for (int b : kSix) HIP_TRY(c, pack1(w.WPp[b], w.W[b], 1.0, 0, 3, 1, 2));
  if (c->crt_moduli) {
    acse_status st = ensure_spin_crt(c, w);
    if (st != ACSE_OK) return st;
    std::vector<const double *> ops;
    for (int b : {B0000, B1111, B0101}) { ops.push_back(w.G2p[b]); ops.push_back(w.Wp[b]); }
    for (int b : kSix) ops.push_back(w.WPp[b]);
    return spin_residues(c, w, r, ops, true);
  }
  return ACSE_OK;
}

// X_A blocks of the residual (X = K): alpha-alpha and beta-beta blocks A_aa,
// the (ab|ab) blocks A_ab = K_s / 2, the (ab|ba) blocks -A_ab with the lower pair exchanged.
acse_status spin_xa_from_fold(acse_ctx c, SpinWs &w, int r) {
  hipStream_t s = c->stream;
  auto comb1 = [&](double *out, const double *in, double coef, int f0, int f1, int f2, int f3) {
    Terms4 T{};
    T.n = 1;
    T.t[0] = term4(in, coef, r, f0, f1, f2, f3);
    return launch_combine4(r, T, out, 0, nullptr, s);
  };
  const double *Aaa = c->ws.Aaa, *Aab = c->ws.Aab;
  HIP_TRY(c, comb1(w.XA[B0000], Aaa, 1.0, 0, 1, 2, 3));
  HIP_TRY(c, comb1(w.XA[B1111], Aaa, 1.0, 0, 1, 2, 3));
  HIP_TRY(c, comb1(w.XA[B0101], Aab, 1.0, 0, 1, 2, 3));
  HIP_TRY(c, comb1(w.XA[B1010], Aab, 1.0, 0, 1, 2, 3));
  HIP_TRY(c, comb1(w.XA[B0110], Aab, -1.0, 0, 1, 3, 2));
  HIP_TRY(c, comb1(w.XA[B1001], Aab, -1.0, 0, 1, 3, 2));
  return ACSE_OK;
}

// X_A blocks of an antisymmetric X given by its three unique blocks.
acse_status spin_xa_from_blocks(acse_ctx c, SpinWs &w, int r, const double *Xaa, const double *Xbb,
                                const double *Xab) {
  hipStream_t s = c->stream;
  auto comb1 = [&](double *out, const double *in, double coef, int f0, int f1, int f2, int f3) {
    Terms4 T{};
    T.n = 1;
    T.t[0] = term4(in, coef, r, f0, f1, f2, f3);
    return launch_combine4(r, T, out, 0, nullptr, s);
  };
  HIP_TRY(c, comb1(w.XA[B0000], Xaa, 1.0, 0, 1, 2, 3));
  HIP_TRY(c, comb1(w.XA[B1111], Xbb, 1.0, 0, 1, 2, 3));
  HIP_TRY(c, comb1(w.XA[B0101], Xab, 1.0, 0, 1, 2, 3));
  HIP_TRY(c, comb1(w.XA[B1010], Xab, 1.0, 1, 0, 3, 2));
  HIP_TRY(c, comb1(w.XA[B0110], Xab, -1.0, 0, 1, 3, 2));
  HIP_TRY(c, comb1(w.XA[B1001], Xab, -1.0, 1, 0, 2, 3));
  return ACSE_OK;
}

// The NY share of the spin-block map: S_b -= C_b for the three output blocks,
// C = B - B(k<->l), B the contraction of X with the NY 3-cumulant of Eq. (8)
// (App. D), over spin-orbital tensors (n = 2r): the block products in FP64,
// or with ACSE_INT8CRT on the int8 matrix cores in exact accumulation, the
// rest in FP64.  The 36 signed
// permutations of the cumulant product collapse by the pair antisymmetry of
// the 2-cumulant and of X's lower pair into
//   B = 4 [sw(t_il) + t_pl - 2 sw(t_ir) - 2 t_pr],  sw(t) = t - t(i<->j),
//   t_il = sum X^{kp}_{rq} c^{ia}_{rq} cs^{jp}_{al},   t_pl = sum Y_ka cs^{ij}_{al},
//   Y_ka = sum X^{kp}_{rq} c^{pa}_{rq},
//   t_ir = sum X^{kp}_{rq} cs^{jp}_{ar} c^{ia}_{lq},   t_pr = sum X^{kp}_{rq} c^{pa}_{lq} cs^{ij}_{ar},
// with c the 2-cumulant and cs = c with its first lower index a weighted by
// sigma_a; each t is two pairwise contractions (n^6 each).  X is the map's
// operator, antisymmetric in both pairs (the X_A blocks).
acse_status ny_spin_share(acse_ctx c, SpinWs &sw, const acse_problem_spin *p, const double *ga, const double *gb) {
  const int r = p->r, n = 2 * r;
  const int64_t n2 = (int64_t)n * n, n3 = n2 * n;
  hipStream_t s = c->stream;
  StageTimer t6(c, 6);
  SoWs *wp = nullptr;
  acse_status st = ensure_so_ws(c, n, 6, wp);
  if (st != ACSE_OK) return st;
  SoWs &w = *wp;
  double *X = w.a[0], *C2 = w.a[1], *CS = w.a[2], *W = w.a[3], *T = w.a[4], *B = w.a[5];
  const bool crt = c->crt_moduli != 0;  // the block products on the int8 matrix cores too
  if ((st = so_upload_sigma(c, w, c->ny_sigma)) != ACSE_OK) return st;
  HIP_TRY(c, launch_fill(n2 * n2, 0.0, X, s));
  for (int b : kSix) HIP_TRY(c, launch_so_embed(r, b, sw.XA[b], 1.0, X, s));
  HIP_TRY(c, launch_so_cumulant(r, ga, gb, p->d2aa, p->d2bb, p->d2ab, w.sig, C2, CS, s));
  // x = i, y = l; then the p, l term through Y
  if ((st = so_contract(c, w, n, W, "kpia", X, "kprq", 1, C2, "iarq", 1, 1.0, 0, crt)) != ACSE_OK) return st;
  HIP_TRY(c, launch_so_trace_y(n, W, w.Y, s));
  if ((st = so_contract(c, w, n, T, "ijkl", W, "kpia", 1, CS, "jpal", 1, 1.0, 0, crt)) != ACSE_OK) return st;
  {
    Terms4 Q{};
    Q.n = 2;
    Q.t[0] = so_term(T, 4.0, n3, n2, n, 1);
    Q.t[1] = so_term(T, -4.0, n2, n3, n, 1);
    HIP_TRY(c, launch_combine4(n, Q, B, 0, nullptr, s));
  }
  HIP_TRY(c, launch_so_tpl(n, 4.0, w.Y, CS, B, s));
  // x = i, y = r (the y = q products equal these)
  if ((st = so_contract(c, w, n, W, "kqja", X, "kprq", 1, CS, "jpar", 1, 1.0, 0, crt)) != ACSE_OK) return st;
  if ((st = so_contract(c, w, n, T, "ijkl", W, "kqja", 3, C2, "ialq", 1, 1.0, 0, crt)) != ACSE_OK) return st;
  {
    Terms4 Q{};
    Q.n = 2;
    Q.t[0] = so_term(T, -8.0, n3, n2, n, 1);
    Q.t[1] = so_term(T, 8.0, n2, n3, n, 1);
    HIP_TRY(c, launch_combine4(n, Q, B, 1, nullptr, s));
  }
  // x = p, y = r: accumulated straight into B
  if ((st = so_contract(c, w, n, W, "kral", X, "kprq", 1, C2, "palq", 1, 1.0, 0, crt)) != ACSE_OK) return st;
  if ((st = so_contract(c, w, n, B, "ijkl", W, "kral", 3, CS, "ijar", 1, -8.0, 1, crt)) != ACSE_OK) return st;
  // S_b -= B_b - B_b(k<->l) on the spin block b of B
  for (int b : {B0000, B1111, B0101}) {
    const int64_t o0 = ((b >> 3) & 1) * (int64_t)r * n3, o1 = ((b >> 2) & 1) * (int64_t)r * n2;
    const int64_t o2 = ((b >> 1) & 1) * (int64_t)r, o3 = (b & 1) * (int64_t)r;
    Terms4 Q{};
    Q.n = 2;
    Q.t[0] = so_term(B + o0 + o1 + o2 * n + o3, -1.0, n3, n2, n, 1);
    Q.t[1] = so_term(B + o0 + o1 + o3 * n + o2, 1.0, n3, n2, 1, n);
    HIP_TRY(c, launch_combine4(r, Q, sw.S[b], 1, nullptr, s));
  }
  return ACSE_OK;
}

// F(X) for the X_A blocks in the workspace into O[0..2] = (aa, bb, ab);
// sigma = -1 Hermitian X, +1 anti-Hermitian.  If Rm is not null it receives
// the masked copy.  The squared block norms land in w.scal[slot .. slot+2].
acse_status spin_map(acse_ctx c, SpinWs &w, const acse_problem_spin *p, const double *ga, const double *gb,
                     double sigma, double *const *O, const ActiveBits *mask, double *const *Rm, int slot) {
  const int r = p->r;
  const int64_t r2 = (int64_t)r * r, r3 = r2 * r;
  const int ld = (int)op_ld(r);
  hipStream_t s = c->stream;
  const double *g[2] = {ga, gb};
  {
    StageTimer t2(c, 2);
    // H = X_A x_1 Gamma1 (index 1 keeps its spin)
    for (int b : {B0000, B1111, B0101, B1001, B0110}) {
      ModeArgs m = mode_base(c, r, g[spin_of(b, 1)]);
      m.A = r; m.Bn = r2; m.in1 = w.XA[b]; m.transpose_m = 1;
      m.so1 = r3; m.so0 = 0; m.sx = r2; m.sb = 1; m.out_cols_fast = 1;
      HIP_TRY(c, launch_mode(GEMM_F64, m, OperandRef{w.H[b], nullptr}, s));
    }
    // f_ks = sum_r H^{kr}_{rs} per spin
    HIP_TRY(c, launch_trace12(r, w.H[B0000], w.f[0], 0, s));
    HIP_TRY(c, launch_trace12(r, w.H[B0110], w.f[0], 1, s));
    HIP_TRY(c, launch_trace12(r, w.H[B1111], w.f[1], 0, s));
    HIP_TRY(c, launch_trace12(r, w.H[B1001], w.f[1], 1, s));
    // t_jk per spin: Gram products over (p, r, s)
    HIP_TRY(c, launch_gram(r, w.W[B0000], w.XA[B0000], 1.0, w.W[B0101], w.XA[B0101], 1.0, w.part, w.t[0], 0, s,
                           c->general));
    HIP_TRY(c, launch_gram(r, w.W[B0110], w.XA[B0110], 1.0, w.W[B0110], w.XA[B0110], 0.0, w.part, w.t[0], 1, s,
                           c->general));
    HIP_TRY(c, launch_gram(r, w.W[B1111], w.XA[B1111], 1.0, w.W[B1010], w.XA[B1010], 1.0, w.part, w.t[1], 0, s,
                           c->general));
    HIP_TRY(c, launch_gram(r, w.W[B1001], w.XA[B1001], 1.0, w.W[B1001], w.XA[B1001], 0.0, w.part, w.t[1], 1, s,
                           c->general));
    // Xt = Gamma1 x_2 X_A (index 2 keeps its spin)
    for (int b : kSix) {
      ModeArgs m = mode_base(c, r, g[spin_of(b, 2)]);
      m.A = r2; m.Bn = r; m.in1 = w.XA[b];
      m.so1 = r2; m.so0 = 0; m.sx = r; m.sb = 1; m.out_cols_fast = 1;
      HIP_TRY(c, launch_mode(GEMM_F64, m, OperandRef{w.Xt[b], nullptr}, s));
    }
    // X-side operands
    auto pack1 = [&](double *out, const double *in, int f0, int f1, int f2, int f3) {
      Terms4 T{};
      T.n = 1;
      T.t[0] = term4(in, 1.0, r, f0, f1, f2, f3);
      return launch_pack_op4(r, T, out, ld, s);
    };
    // same-spin X_A and H: rows (k,l), K r < s (both antisymmetric in (r,s))
    for (int b : {B0000, B1111}) {
      HIP_TRY(c, launch_spin_pack_lt(r, w.XA[b], 1.0, 0, w.XAp[b], s));
      HIP_TRY(c, launch_spin_pack_lt(r, w.H[b], 1.0, 0, w.Hp[b], s));
    }
    HIP_TRY(c, pack1(w.XAp[B0101], w.XA[B0101], 0, 1, 2, 3));
    for (int b : {B0101, B1001}) HIP_TRY(c, pack1(w.Hp[b], w.H[b], 0, 1, 2, 3));
    for (int b : kSix) HIP_TRY(c, pack1(w.XtP[b], w.Xt[b], 0, 2, 1, 3));  // rows (k,i), K (p,s)
    if (c->crt_moduli) {
      std::vector<const double *> ops;
      for (int b : {B0000, B1111, B0101}) ops.push_back(w.XAp[b]);
      for (int b : {B0000, B1111, B0101, B1001}) ops.push_back(w.Hp[b]);
      for (int b : kSix) ops.push_back(w.XtP[b]);
      acse_status st = spin_residues(c, w, r, ops, false);
      if (st != ACSE_OK) return st;
    }
  }
  // the 17 products in three launches of 6, 6 and 5; the second E term of the
  // four blocks that have one accumulates in the last launch, after the
  // launch that wrote the first.  The same-spin Y and W H products run over
  // the pairs i < j and r < s (a quarter of the flops; alpha doubled for the
  // summed pair) into row-major scratch, unpacked afterwards.
  {
    const int kp = gemm_kp(GEMM_F64, (int)r2, ld);
    auto prob = [&](GemmProb &P, const double *A, const double *B, double alpha, double *C, bool ph, int acc) {
      P = GemmProb{};
      P.A = A; P.B = B; P.C = C; P.alpha = alpha;
      P.M = (int)r2; P.N = (int)r2; P.Kp = kp; P.ld = ld; P.rdiv = r;
      if (ph) { P.sm1 = r; P.sm0 = r3; P.sn1 = r2; P.sn0 = 1; }      // rows (k,i), cols (j,l) -> [i,j,k,l]
      else { P.sm1 = r3; P.sm0 = r2; P.sn1 = r; P.sn0 = 1; }         // natural [(ij)][(kl)]
      P.ksplit = 1; P.kchunk = kp; P.accumulate = acc;
    };
    const int nlt = npair_lt(r);
    const int64_t ldlt = ld_pair_lt(r);
    auto probp = [&](GemmProb &P, const double *A, const double *B, double alpha, double *C) {
      P = GemmProb{};
      P.A = A; P.B = B; P.C = C; P.alpha = alpha;
      P.M = nlt; P.N = (int)r2; P.Kp = gemm_kp(GEMM_F64, nlt, (int)ldlt); P.ld = (int)ldlt; P.rdiv = 1;
      P.sm1 = r2; P.sm0 = 0; P.sn1 = 1; P.sn0 = 0;                   // row-major [pairs][r^2]
      P.ksplit = 1; P.kchunk = P.Kp; P.accumulate = 0;
    };
    const int cfg = map_cfg(c, GEMM_F64, r, -1);
    // FP64 products, or the int8 exact-accumulation ones from the residues of
    // the same operand buffers (the reconstruction writes through the same
    // store maps)
    auto launch = [&](GemmBatch &b) -> acse_status {
      if (!c->crt_moduli) {
        StageTimer t3(c, 3);
        HIP_TRY(c, gemm_launch(GEMM_F64, cfg, b, s));
        return ACSE_OK;
      }
      int64_t yoff = 0;
      for (int q = 0; q < b.count; ++q) {
        GemmProb &P = b.p[q];
        const int ka = spin_op_index(w, static_cast<const double *>(P.A));
        const int kb = spin_op_index(w, static_cast<const double *>(P.B));
        if (ka < 0 || kb < 0) return fail(c, ACSE_ERR_HIP, "internal: unknown spin operand buffer");
        const int K = spin_op_shape(w, static_cast<const double *>(P.A), r).K;
        P.A = w.cres[ka];
        P.B = w.cres[kb];
        P.ld = P.Kp = (int)crt_ldr(K);
        P.kchunk = P.Kp;
        P.plane_a = P.plane_b = op_rows(r) * crt_ldr(K);
        P.ea = w.cexp[ka];
        P.eb = w.cexp[kb];
        P.kshift = 2 * crt_kbits(c->crt, K);
        P.Y = w.cy + yoff;
        P.plane_y = crt_residue_out_bytes(P.M, P.N);
        yoff += (int64_t)c->crt.nmod * P.plane_y;
      }
      {
        StageTimer t3(c, 3);
        HIP_TRY(c, gemm_crt_launch(b, c->crt, s));
      }
      StageTimer t4(c, 4);
      HIP_TRY(c, crt_combine_launch(b, c->crt, s));
      return ACSE_OK;
    };
    acse_status st;
    GemmBatch b1{};
    b1.count = 6;
    probp(b1.p[0], w.G2p[B0000], w.XAp[B0000], 2.0, w.Pk[0]);
    probp(b1.p[1], w.G2p[B1111], w.XAp[B1111], 2.0, w.Pk[1]);
    prob(b1.p[2], w.G2p[B0101], w.XAp[B0101], 2.0, w.Y[B0101], false, 0);
    probp(b1.p[3], w.Wp[B0000], w.Hp[B0000], 2.0, w.Pk[2]);
    probp(b1.p[4], w.Wp[B1111], w.Hp[B1111], 2.0, w.Pk[3]);
    prob(b1.p[5], w.Wp[B0101], w.Hp[B0101], 2.0, w.T[B0101], false, 0);
    if ((st = launch(b1)) != ACSE_OK) return st;
    {
      StageTimer t4(c, 4);
      double *const dst[4] = {w.Y[B0000], w.Y[B1111], w.T[B0000], w.T[B1111]};
      for (int k = 0; k < 4; ++k) HIP_TRY(c, launch_unpack_rows_lt(r, w.Pk[k], r2, dst[k], s));
    }
    // E^{ij}_{kl} = 2 sum Xt^{kp}_{is} W^{jp}_{sl}: the first terms of the four
    // blocks with two, then the rest
    GemmBatch b2{};
    b2.count = 6;
    prob(b2.p[0], w.Wp[B0101], w.Hp[B1001], 2.0, w.T[B0110], false, 0);
    prob(b2.p[1], w.XtP[B0000], w.WPp[B0000], 2.0, w.E[B0000], true, 0);
    prob(b2.p[2], w.XtP[B1111], w.WPp[B1111], 2.0, w.E[B1111], true, 0);
    prob(b2.p[3], w.XtP[B0000], w.WPp[B1001], 2.0, w.E[B0101], true, 0);
    prob(b2.p[4], w.XtP[B1010], w.WPp[B0000], 2.0, w.E[B1010], true, 0);
    prob(b2.p[5], w.XtP[B0110], w.WPp[B0101], 2.0, w.E[B1001], true, 0);
    if ((st = launch(b2)) != ACSE_OK) return st;
    GemmBatch b3{};
    b3.count = 5;
    prob(b3.p[0], w.XtP[B1001], w.WPp[B1010], 2.0, w.E[B0110], true, 0);
    prob(b3.p[1], w.XtP[B0101], w.WPp[B0110], 2.0, w.E[B0000], true, 1);
    prob(b3.p[2], w.XtP[B1010], w.WPp[B1001], 2.0, w.E[B1111], true, 1);
    prob(b3.p[3], w.XtP[B0101], w.WPp[B1111], 2.0, w.E[B0101], true, 1);
    prob(b3.p[4], w.XtP[B1111], w.WPp[B0110], 2.0, w.E[B1010], true, 1);
    if ((st = launch(b3)) != ACSE_OK) return st;
  }
  StageTimer t4(c, 4);
  // T += 2 sum_s f_ks W^{ij}_{sl} (index 2 of W keeps its spin)
  for (int b : {B0000, B1111, B0101, B0110}) {
    ModeArgs m = mode_base(c, r, w.f[spin_of(b, 2)]);
    m.A = r2; m.Bn = r; m.in1 = w.W[b]; m.alpha = 2.0; m.accumulate = 1;
    m.so1 = r2; m.so0 = 0; m.sx = r; m.sb = 1; m.out_cols_fast = 1;
    HIP_TRY(c, launch_mode(GEMM_F64, m, OperandRef{w.T[b], nullptr}, s));
  }
  // T += Gamma1_il t_jk - Gamma1_jl t_ik
  HIP_TRY(c, launch_outer4(r, 1.0, ga, 0, 3, w.t[0], 1, 2, w.T[B0000], s));
  HIP_TRY(c, launch_outer4(r, -1.0, ga, 1, 3, w.t[0], 0, 2, w.T[B0000], s));
  HIP_TRY(c, launch_outer4(r, 1.0, gb, 0, 3, w.t[1], 1, 2, w.T[B1111], s));
  HIP_TRY(c, launch_outer4(r, -1.0, gb, 1, 3, w.t[1], 0, 2, w.T[B1111], s));
  HIP_TRY(c, launch_outer4(r, -1.0, gb, 1, 3, w.t[0], 0, 2, w.T[B0101], s));
  HIP_TRY(c, launch_outer4(r, 1.0, ga, 0, 3, w.t[1], 1, 2, w.T[B0110], s));
  // S = Y - C, C = T' - T'(k<->l), T' = T + E - E(i<->j)
  struct Sel { int b, bl, bi, bli; };  // block, its k<->l partner, i<->j of each
  const Sel sel[3] = {{B0000, B0000, B0000, B0000}, {B1111, B1111, B1111, B1111}, {B0101, B0110, B1001, B1010}};
  const int out_blocks[3] = {B0000, B1111, B0101};
  for (int q = 0; q < 3; ++q) {
    const Sel &x = sel[q];
    Terms4 T{};
    T.n = 7;
    T.t[0] = term4(w.Y[x.b], 1.0, r, 0, 1, 2, 3);
    T.t[1] = term4(w.T[x.b], -1.0, r, 0, 1, 2, 3);
    T.t[2] = term4(w.E[x.b], -1.0, r, 0, 1, 2, 3);
    T.t[3] = term4(w.E[x.bi], 1.0, r, 1, 0, 2, 3);
    T.t[4] = term4(w.T[x.bl], 1.0, r, 0, 1, 3, 2);
    T.t[5] = term4(w.E[x.bl], 1.0, r, 0, 1, 3, 2);
    T.t[6] = term4(w.E[x.bli], -1.0, r, 1, 0, 3, 2);
    HIP_TRY(c, launch_combine4(r, T, w.S[out_blocks[q]], 0, nullptr, s));
  }
  t4.stop();
  if (c->ny_on) {
    acse_status st = ny_spin_share(c, w, p, ga, gb);
    if (st != ACSE_OK) return st;
  }
  StageTimer t4b(c, 4);
  // F = S + sigma S^T, the masked copy, the block norms
  for (int q = 0; q < 3; ++q) {
    const int b = out_blocks[q];
    Terms4 T{};
    T.n = 2;
    T.t[0] = term4(w.S[b], 1.0, r, 0, 1, 2, 3);
    T.t[1] = term4(w.S[b], sigma, r, 2, 3, 0, 1);
    HIP_TRY(c, launch_combine4(r, T, O[q], 0, nullptr, s));
    if (Rm) {
      Terms4 M{};
      M.n = 1;
      M.t[0] = term4(O[q], 1.0, r, 0, 1, 2, 3);
      HIP_TRY(c, launch_combine4(r, M, Rm[q], 0, mask, s));
    }
    HIP_TRY(c, launch_dot(r2 * r2, O[q], O[q], w.part, w.scal + slot + q, s));
  }
  return ACSE_OK;
}

// Host copies of n scalars from w.scal (synchronises).
acse_status spin_fetch(acse_ctx c, SpinWs &w, double *host, int n) {
  HIP_TRY(c, hipMemcpyAsync(host, w.scal, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return ACSE_OK;
}

acse_status spin_energy(acse_ctx c, SpinWs &w, const acse_problem_spin *p, int slot) {
  // E = <K_s, d2aa> + <K_s, d2bb> + 2 <K_s, d2ab>, K_s = 2 A_ab (the fold's unantisymmetrised half)
  const int64_t n4 = (int64_t)p->r * p->r * p->r * p->r;
  HIP_TRY(c, launch_dot(n4, c->ws.Aab, p->d2aa, w.part, w.scal + slot, c->stream));
  HIP_TRY(c, launch_dot(n4, c->ws.Aab, p->d2bb, w.part, w.scal + slot + 1, c->stream));
  HIP_TRY(c, launch_dot(n4, c->ws.Aab, p->d2ab, w.part, w.scal + slot + 2, c->stream));
  return ACSE_OK;
}

acse_status spin_check_outputs(acse_ctx c, std::initializer_list<const void *> outs) {
  for (const void *q : outs)
    if (q && !aligned16(q)) return fail(c, ACSE_ERR_ALIGN, "output arrays must be 16-byte aligned");
  return ACSE_OK;
}

}  // namespace

extern "C" acse_status acse_energy_spin(acse_ctx ctx, const acse_problem_spin *prob, double *E_host) {
  acse_status st = validate_spin(ctx, prob, nullptr, false);
  if (st != ACSE_OK) return st;
  if (!E_host) return fail(ctx, ACSE_ERR_ARG, "E_host is NULL");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  SpinWs *w = nullptr;
  if ((st = ensure_spin_ws(ctx, w)) != ACSE_OK) return st;
  HIP_TRY(ctx, launch_fold(prob->r, prob->n_alpha + prob->n_beta, prob->h, prob->V, ctx->ws.Aaa, ctx->ws.Aab,
                           ctx->stream));
  if ((st = spin_energy(ctx, *w, prob, 0)) != ACSE_OK) return st;
  double e[3];
  if ((st = spin_fetch(ctx, *w, e, 3)) != ACSE_OK) return st;
  *E_host = 2.0 * (e[0] + e[1]) + 4.0 * e[2];
  if (!std::isfinite(*E_host)) return fail(ctx, ACSE_ERR_NONFINITE, "energy is not finite");
  return ACSE_OK;
}

extern "C" acse_status acse_residual_spin(acse_ctx ctx, const acse_problem_spin *prob, const acse_options *opts,
                                          double *R_aa, double *R_bb, double *R_ab, double *norm2_host) {
  acse_status st = validate_spin(ctx, prob, opts, true);
  if (st != ACSE_OK) return st;
  for (auto q : {std::make_pair((const void *)R_aa, "R_aa"), std::make_pair((const void *)R_bb, "R_bb"),
                 std::make_pair((const void *)R_ab, "R_ab")})
    if ((st = check_out(ctx, q.first, q.second)) != ACSE_OK) return st;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  SpinWs *w = nullptr;
  if ((st = ensure_spin_ws(ctx, w)) != ACSE_OK) return st;
  const int r = prob->r;
  if ((st = spin_prep(ctx, *w, prob)) != ACSE_OK) return st;
  {
    StageTimer t1(ctx, 1);
    HIP_TRY(ctx, launch_fold(r, prob->n_alpha + prob->n_beta, prob->h, prob->V, ctx->ws.Aaa, ctx->ws.Aab,
                             ctx->stream));
  }
  if ((st = spin_xa_from_fold(ctx, *w, r)) != ACSE_OK) return st;
  double *O[3] = {R_aa, R_bb, R_ab};
  if ((st = spin_map(ctx, *w, prob, prob->d1a, prob->d1b, -1.0, O, nullptr, nullptr, 0)) != ACSE_OK) return st;
  if (!norm2_host) return ACSE_OK;
  double n[3];
  if ((st = spin_fetch(ctx, *w, n, 3)) != ACSE_OK) return st;
  *norm2_host = n[0] + n[1] + 4.0 * n[2];
  if (!std::isfinite(*norm2_host)) return fail(ctx, ACSE_ERR_NONFINITE, "||R||^2 is not finite");
  return ACSE_OK;
}

extern "C" acse_status acse_step_spin(acse_ctx ctx, acse_problem_spin *prob, double eps, const acse_options *opts,
                                      double *R_aa, double *R_bb, double *R_ab, double *U_aa, double *U_bb,
                                      double *U_ab, double *E_host, double *norm2_host) {
  acse_status st = validate_spin(ctx, prob, opts, true);
  if (st != ACSE_OK) return st;
  if (!std::isfinite(eps)) return fail(ctx, ACSE_ERR_ARG, "eps is not finite");
  if ((st = spin_check_outputs(ctx, {R_aa, R_bb, R_ab, U_aa, U_bb, U_ab})) != ACSE_OK) return st;
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  SpinWs *w = nullptr;
  if ((st = ensure_spin_ws(ctx, w)) != ACSE_OK) return st;
  const int r = prob->r;
  const int N = prob->n_alpha + prob->n_beta;
  hipStream_t s = ctx->stream;
  double *R[3] = {R_aa ? R_aa : w->R[0], R_bb ? R_bb : w->R[1], R_ab ? R_ab : w->R[2]};
  double *U[3] = {U_aa ? U_aa : w->U[0], U_bb ? U_bb : w->U[1], U_ab ? U_ab : w->U[2]};
  bool masked = false;
  const ActiveBits act = make_bits(opts, r, &masked);
  if ((st = spin_prep(ctx, *w, prob)) != ACSE_OK) return st;
  {
    StageTimer t1(ctx, 1);
    HIP_TRY(ctx, launch_fold(r, N, prob->h, prob->V, ctx->ws.Aaa, ctx->ws.Aab, s));
  }
  if ((st = spin_xa_from_fold(ctx, *w, r)) != ACSE_OK) return st;
  // R = F(K), block norms -> scal[0..2], masked copy
  if ((st = spin_map(ctx, *w, prob, prob->d1a, prob->d1b, -1.0, R, masked ? &act : nullptr, masked ? w->Rm : nullptr,
                     0)) != ACSE_OK)
    return st;
  // U = F(R_m) on the same 2-RDM
  const double *const *Xm = masked ? w->Rm : R;
  if ((st = spin_xa_from_blocks(ctx, *w, r, Xm[0], Xm[1], Xm[2])) != ACSE_OK) return st;
  if ((st = spin_map(ctx, *w, prob, prob->d1a, prob->d1b, 1.0, U, nullptr, nullptr, 3)) != ACSE_OK) return st;
  // 2D <- (2D + eps U) per block at its input trace; 1-RDM per spin; energy
  {
    StageTimer t5(ctx, 5);
    const double *tr_in[6] = {prob->d2aa, prob->d2bb, prob->d2ab, U[0], U[1], U[2]};
    double *traces = w->scal + 16;
    HIP_TRY(ctx, launch_pair_traces(r, 6, tr_in, traces, s));
    double *d2[3] = {prob->d2aa, prob->d2bb, prob->d2ab};
    const double *Uc[3] = {U[0], U[1], U[2]};
    HIP_TRY(ctx, launch_spin_update(r, eps, d2, Uc, traces, s));
    HIP_TRY(ctx, launch_spin_1rdm(r, N, prob->d2aa, prob->d2bb, prob->d2ab, prob->d1a, prob->d1b, s));
    if ((st = spin_energy(ctx, *w, prob, 6)) != ACSE_OK) return st;
  }
  if (!E_host && !norm2_host) return ACSE_OK;
  double v[9];
  if ((st = spin_fetch(ctx, *w, v, 9)) != ACSE_OK) return st;
  if (norm2_host) {
    *norm2_host = v[0] + v[1] + 4.0 * v[2];
    if (!std::isfinite(*norm2_host)) return fail(ctx, ACSE_ERR_NONFINITE, "||R||^2 is not finite");
  }
  if (E_host) {
    *E_host = 2.0 * (v[6] + v[7]) + 4.0 * v[8];
    if (!std::isfinite(*E_host)) return fail(ctx, ACSE_ERR_NONFINITE, "energy is not finite");
  }
  return ACSE_OK;
}

// Euler iteration of a state of any S_z: the driver of acse_solve with the
// spin-block residual map, the per-block trace restoration and the 1-RDM per
// spin (FIXED and BACKTRACK controls).
extern "C" acse_status acse_solve_spin(acse_ctx ctx, acse_problem_spin *prob, const acse_options *opts,
                                       const acse_solve_options *so, acse_solve_result *res, acse_trial *hist,
                                       int32_t cap) {
  acse_status st = validate_spin(ctx, prob, opts, true);
  if (st != ACSE_OK) return st;
  if ((st = check_solve_options(ctx, so, res, hist, cap)) != ACSE_OK) return st;
  const bool quad = so->control == ACSE_EULER_QUADRATIC;
  const double eps_max = so->eps_max > 0.0 ? so->eps_max : 16.0 * std::fabs(so->eps);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  SpinWs *wp = nullptr;
  if ((st = ensure_spin_ws(ctx, wp)) != ACSE_OK) return st;
  SpinWs &w = *wp;
  if (quad && !w.qbase) {
    const int64_t rm2 = (int64_t)ctx->r_max * ctx->r_max;
    const int64_t nat = round_up(rm2 * rm2 * 8, 256), sm = round_up(rm2 * 8, 256);
    if (hipMalloc(&w.qbase, 6 * nat + 2 * sm) != hipSuccess) {
      (void)hipGetLastError();
      w.qbase = nullptr;
      return fail(ctx, ACSE_ERR_NOMEM, "cannot allocate the workspace of the quadratic control");
    }
    char *q = static_cast<char *>(w.qbase);
    for (int k = 0; k < 3; ++k, q += nat) w.Rk[k] = reinterpret_cast<double *>(q);
    for (int k = 0; k < 3; ++k, q += nat) w.Qa[k] = reinterpret_cast<double *>(q);
    for (int k = 0; k < 2; ++k, q += sm) w.dg[k] = reinterpret_cast<double *>(q);
  }
  if (ctx->crt_moduli && (st = ensure_spin_crt(ctx, w)) != ACSE_OK) return st;
  if (!w.kbase) {
    const int64_t rm2 = (int64_t)ctx->r_max * ctx->r_max;
    const int64_t nat = round_up(rm2 * rm2 * 8, 256), sm = round_up(rm2 * 8, 256);
    if (hipMalloc(&w.kbase, 3 * nat + 2 * sm) != hipSuccess) {
      (void)hipGetLastError();
      w.kbase = nullptr;
      return fail(ctx, ACSE_ERR_NOMEM, "cannot allocate the spin-block driver workspace");
    }
    char *q = static_cast<char *>(w.kbase);
    for (int k = 0; k < 3; ++k, q += nat) w.Nk[k] = reinterpret_cast<double *>(q);
    for (int k = 0; k < 2; ++k, q += sm) w.gk[k] = reinterpret_cast<double *>(q);
  }
  hipStream_t s = ctx->stream;
  const int r = prob->r;
  const int N = prob->n_alpha + prob->n_beta;
  const int64_t r2 = (int64_t)r * r, n4 = r2 * r2;
  bool masked = false;
  const ActiveBits act = make_bits(opts, r, &masked);
  double *d2[3] = {prob->d2aa, prob->d2bb, prob->d2ab};
  double *d1[2] = {prob->d1a, prob->d1b};
  double *traces = w.scal + 16;  // input traces of 2D_n's blocks, then U_n's

  *res = acse_solve_result{};
  auto record = [&](double x, double E, double f, int n) -> int32_t {
    const int32_t id = res->trials++;
    if (id < cap) hist[id] = acse_trial{x, E, f, n, 0};
    return id;
  };
  auto mark = [&](int32_t id) { if (id >= 0 && id < cap) hist[id].accepted = 1; };
  // residual of the problem arrays into w.R (masked copy into w.Rm), its
  // ||R||^2 and the energy; the map's operands of this state stay in place
  auto residual = [&](double *f, double *E) -> acse_status {
    acse_status q;
    if ((q = spin_prep(ctx, w, prob)) != ACSE_OK) return q;
    if ((q = spin_xa_from_fold(ctx, w, r)) != ACSE_OK) return q;
    if ((q = spin_map(ctx, w, prob, prob->d1a, prob->d1b, -1.0, w.R, masked ? &act : nullptr,
                      masked ? w.Rm : nullptr, 0)) != ACSE_OK)
      return q;
    ++res->maps;
    if ((q = spin_energy(ctx, w, prob, 6)) != ACSE_OK) return q;
    double v[9];
    if ((q = spin_fetch(ctx, w, v, 9)) != ACSE_OK) return q;
    *f = v[0] + v[1] + 4.0 * v[2];
    *E = 2.0 * (v[6] + v[7]) + 4.0 * v[8];
    if (!std::isfinite(*f)) return fail(ctx, ACSE_ERR_NONFINITE, "||R||^2 is not finite");
    if (!std::isfinite(*E)) return fail(ctx, ACSE_ERR_NONFINITE, "energy is not finite");
    return ACSE_OK;
  };
  auto restore = [&](bool with_1rdm) -> acse_status {
    for (int k = 0; k < 3; ++k) HIP_TRY(ctx, hipMemcpyAsync(d2[k], w.Nk[k], n4 * 8, hipMemcpyDeviceToDevice, s));
    if (with_1rdm)
      for (int k = 0; k < 2; ++k) HIP_TRY(ctx, hipMemcpyAsync(d1[k], w.gk[k], r2 * 8, hipMemcpyDeviceToDevice, s));
    return ACSE_OK;
  };
  // trial: each block of (2D_n + x U_n) at 2D_n's trace, the 1-RDMs contracted
  // from it, E' and ||R'||^2
  auto trial = [&](double x, bool from_kept, double *f, double *E) -> acse_status {
    acse_status q;
    if (from_kept && (q = restore(false)) != ACSE_OK) return q;
    {
      StageTimer t5(ctx, 5);
      const double *Uc[3] = {w.U[0], w.U[1], w.U[2]};
      HIP_TRY(ctx, launch_spin_update(r, x, d2, Uc, traces, s));
      HIP_TRY(ctx, launch_spin_1rdm(r, N, prob->d2aa, prob->d2bb, prob->d2ab, prob->d1a, prob->d1b, s));
    }
    return residual(f, E);
  };

  {
    StageTimer t1(ctx, 1);
    HIP_TRY(ctx, launch_fold(r, N, prob->h, prob->V, ctx->ws.Aaa, ctx->ws.Aab, s));
  }
  double E = 0.0, f = 0.0;
  if ((st = residual(&f, &E)) != ACSE_OK) return st;
  res->energy0 = res->energy = E;
  res->norm2_0 = res->norm2 = f;
  res->stop = ACSE_STOP_MAX_ITER;
  double e = so->eps;

  for (int n = 0; n < so->max_iter; ++n) {
    // U_n = F(R_m) on the operands of 2D_n (left in place by its residual)
    const double *const *Xm = masked ? w.Rm : w.R;
    if ((st = spin_xa_from_blocks(ctx, w, r, Xm[0], Xm[1], Xm[2])) != ACSE_OK) return st;
    if ((st = spin_map(ctx, w, prob, prob->d1a, prob->d1b, 1.0, w.U, nullptr, nullptr, 3)) != ACSE_OK) return st;
    ++res->maps;
    // keep 2D_n and 1D_n; the block traces the trials restore
    for (int k = 0; k < 3; ++k) HIP_TRY(ctx, hipMemcpyAsync(w.Nk[k], d2[k], n4 * 8, hipMemcpyDeviceToDevice, s));
    for (int k = 0; k < 2; ++k) HIP_TRY(ctx, hipMemcpyAsync(w.gk[k], d1[k], r2 * 8, hipMemcpyDeviceToDevice, s));
    {
      const double *tr_in[6] = {d2[0], d2[1], d2[2], w.U[0], w.U[1], w.U[2]};
      HIP_TRY(ctx, launch_pair_traces(r, 6, tr_in, traces, s));
    }
    // f'(0) of f(x) = ||R(2D_n + x U_n, 1D_n + x dD)||^2, dD the 1-RDMs
    // contracted from U_n: along this line R is a polynomial of degree at
    // most 4 in x (the 3-RDM is at most quartic in the RDMs), so the
    // five-point central difference of R at x = +-h, +-2h (h = eps) is its
    // exact derivative up to rounding; f'(0) = 2 <R_n, R'(0)> over spin
    // orbitals.  The trace restoration of the trials leaves the slope
    // unchanged (Tr U_n = 0 per block).
    double g0 = 0.0;
    if (quad) {
      for (int k = 0; k < 3; ++k) {
        HIP_TRY(ctx, hipMemcpyAsync(w.Rk[k], w.R[k], n4 * 8, hipMemcpyDeviceToDevice, s));
        HIP_TRY(ctx, launch_fill(n4, 0.0, w.Qa[k], s));
      }
      HIP_TRY(ctx, launch_spin_1rdm(r, N, w.U[0], w.U[1], w.U[2], w.dg[0], w.dg[1], s));
      const double h = e;
      const double xs[4] = {h, -h, 2.0 * h, -2.0 * h}, cw[4] = {8.0, -8.0, -1.0, 1.0};
      for (int q = 0; q < 4; ++q) {
        for (int k = 0; k < 3; ++k) HIP_TRY(ctx, launch_spin_axpy(n4, w.Nk[k], xs[q], w.U[k], d2[k], s));
        for (int k = 0; k < 2; ++k) HIP_TRY(ctx, launch_spin_axpy(r2, w.gk[k], xs[q], w.dg[k], d1[k], s));
        double fq = 0.0, Eq = 0.0;
        if ((st = residual(&fq, &Eq)) != ACSE_OK) return st;
        for (int k = 0; k < 3; ++k) HIP_TRY(ctx, launch_spin_axpy(n4, w.Qa[k], cw[q], w.R[k], w.Qa[k], s));
      }
      for (int k = 0; k < 3; ++k) HIP_TRY(ctx, launch_dot(n4, w.Rk[k], w.Qa[k], w.part, w.scal + 32 + k, s));
      double dots[3];
      HIP_TRY(ctx, hipMemcpyAsync(dots, w.scal + 32, sizeof dots, hipMemcpyDeviceToHost, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
      g0 = 2.0 * (dots[0] + dots[1] + 4.0 * dots[2]) / (12.0 * h);
      if (!std::isfinite(g0)) return fail(ctx, ACSE_ERR_NONFINITE, "slope of ||R||^2 is not finite");
    }

    auto ok = [&](double Et, double ft) { return Et <= E && ft <= f; };
    const double x1 = e;
    double xc = x1, fc = 0.0, Ec = 0.0;
    // the slope's evaluations left the line's last point in the arrays
    if ((st = trial(xc, quad, &fc, &Ec)) != ACSE_OK) return st;
    int32_t idc = record(xc, Ec, fc, n);
    const double f1 = fc, E1 = Ec;
    const int32_t id1 = idc;
    bool chosen = ok(Ec, fc);
    double last_E = Ec;
    double cand = e;
    if (quad) {
      const double x2 = quadratic_second_step(f, g0, x1, f1, eps_max);
      if (x2 != 0.0) {
        double f2 = 0.0, E2 = 0.0;
        if ((st = trial(x2, true, &f2, &E2)) != ACSE_OK) return st;
        const int32_t id2 = record(x2, E2, f2, n);
        last_E = E2;
        const bool ok1 = ok(E1, f1), ok2 = ok(E2, f2);
        if (ok2 && (!ok1 || f2 < f1)) {
          chosen = true; xc = x2; fc = f2; Ec = E2; idc = id2;
        } else if (ok1) {
          // the arrays hold the second trial: evaluate the first again (same kernels, same values)
          double fr = 0.0, Er = 0.0;
          if ((st = trial(x1, true, &fr, &Er)) != ACSE_OK) return st;
          chosen = true; xc = x1; fc = f1; Ec = E1; idc = id1;
        } else {
          chosen = false;
        }
        cand = std::min(x1, x2);
      }
    }
    for (int hv = 0; !chosen && so->control != ACSE_EULER_FIXED && hv < so->max_halvings; ++hv) {
      cand *= 0.5;
      double ft = 0.0, Et = 0.0;
      if ((st = trial(cand, true, &ft, &Et)) != ACSE_OK) return st;
      const int32_t id = record(cand, Et, ft, n);
      last_E = Et;
      if (ok(Et, ft)) { chosen = true; xc = cand; fc = ft; Ec = Et; idc = id; }
    }
    if (!chosen) {
      // keep the state before the rise
      if ((st = restore(true)) != ACSE_OK) return st;
      HIP_TRY(ctx, hipStreamSynchronize(s));
      res->stop = last_E > E ? ACSE_STOP_ENERGY_ROSE : ACSE_STOP_NORM_ROSE;
      break;
    }
    mark(idc);
    const double dE = Ec - E;
    E = Ec;
    f = fc;
    e = xc;
    res->iterations = n + 1;
    res->eps = xc;
    res->energy = E;
    res->norm2 = f;
    if (std::fabs(dE) < so->de_tol) {
      res->stop = ACSE_STOP_CONVERGED;
      break;
    }
  }
  return ACSE_OK;
}

namespace {
void release_spin_ws(acse_ctx c) {
  SpinWs *w = static_cast<SpinWs *>(c->spws);
  if (w && w->cbase) (void)hipFree(w->cbase);
  if (w && w->kbase) (void)hipFree(w->kbase);
  if (w && w->qbase) (void)hipFree(w->qbase);
  delete w;
  c->spws = nullptr;
}
}  // namespace
