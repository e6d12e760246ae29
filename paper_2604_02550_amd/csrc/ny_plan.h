// Spin-block plan of the Nakatsuji-Yasuda share of the residual map (host
// only, no HIP).
//
// The NY 3-cumulant (Eq. (8); App. D, NY part) enters F(X) only through
// B^{ij}_{kl} = 6 sum_pqr X^{kp}_{rq} 3Delta^{ijp}_{rql}.  With X and the
// 2-cumulant Delta antisymmetric in both index pairs, the 36 signed
// permutations collapse to
//   B = 4 [ sw(T_il) + T_pl - 2 sw(T_ir) - 2 T_pr ],  sw(T)^{ij}_{kl} = T^{ij}_{kl} - T^{ji}_{kl},
//   T_il = sum_{pa} W[i,k,p,a] sD^{jp}_{al},   W[i,k,p,a] = sum_{rq} X^{kp}_{rq} D^{ia}_{rq}
//   T_ir = sum_{qa} Z[k,j,q,a] D^{ia}_{lq},    Z[k,j,q,a] = sum_{pr} X^{kp}_{rq} sD^{jp}_{ar}
//   T_pr = sum_{ra} V[k,l,r,a] sD^{ij}_{ar},   V[k,l,r,a] = sum_{pq} X^{kp}_{rq} D^{pa}_{lq}
//   T_pl = sum_a Y[k,a] sD^{ij}_{al},          Y[k,a]     = sum_p W[p,k,p,a]
// with sD^{..}_{a.} = sigma_a D^{..}_{a.} (the third index scaled).  The
// y = q products of the nine equal the y = r ones by the antisymmetry of X in
// its lower pair.
//
// Every tensor is a spin-orbital one held as spatial blocks: block b of a
// 4-index tensor has bit (3 - t) set when index t is beta.  For singlet
// inputs a tensor equals itself with all spins flipped, so only blocks with
// index 0 alpha (b < 8) are stored ("canonical"); block b ^ 15 is the same
// array.  The inputs X, D, sD have the canonical blocks 0000 (alpha-alpha),
// 0101 (alpha-beta) and 0110 (= minus the alpha-beta block with its last two
// indices exchanged); every other block is zero.
//
// Each two-index-pair contraction is a sum, over the spins of its internal
// indices, of r^2 x r^2 x r^2 products of spatial blocks.  The planner
// enumerates the spin assignments, keeps the canonical output blocks the
// final combination needs (and those the first stages must produce for
// them), and emits permutations of source blocks into GEMM operand layout and
// the GEMM list.
#pragma once
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

namespace acse {
namespace ny {

// Tensors of the plan.  Sources: natural r^4 arrays per canonical block.
// Intermediates: stored in the next stage's GEMM operand layout (rows = the
// first two letters of their storage order, K = the last two).  Products:
// natural r^4 arrays [i,j,k,l] per canonical block.
enum Tensor { T_X = 0, T_D, T_SD, T_W, T_Z, T_V, T_IL, T_IR, T_PR, kNumTensors };

inline bool is_source(int t) { return t <= T_SD; }
inline bool is_product(int t) { return t >= T_IL; }

struct Stage {
  int a, b, out;
  const char *la, *ra, *ka;  // A: natural letters, GEMM row letters, K letters
  const char *lb, *rb, *kb;  // B: the same (K letters in the same order as A's)
  const char *lo;            // output storage letters
};

// First-stage products, then the second stages (which read them).
inline const Stage *stages(int *count) {
  static const Stage s[6] = {
      {T_X, T_D, T_W, "kprq", "kp", "rq", "iarq", "ia", "rq", "ikpa"},
      {T_X, T_SD, T_Z, "kprq", "kq", "pr", "jpar", "ja", "pr", "kjqa"},
      {T_X, T_D, T_V, "kprq", "kr", "pq", "palq", "al", "pq", "klra"},
      {T_W, T_SD, T_IL, "ikpa", "ik", "pa", "jpal", "jl", "pa", "ijkl"},
      {T_Z, T_D, T_IR, "kjqa", "kj", "qa", "ialq", "il", "qa", "ijkl"},
      {T_V, T_SD, T_PR, "klra", "kl", "ra", "ijar", "ij", "ra", "ijkl"},
  };
  *count = 6;
  return s;
}

inline int canon(int b) { return (b & 8) ? (b ^ 15) : b; }
inline bool source_nonzero(int b) {
  const int c = canon(b);
  return c == 0 || c == 5 || c == 6;
}
// canonical product blocks the final combination reads
inline const int *product_blocks(int *count) {
  static const int b[3] = {0, 5, 6};
  *count = 3;
  return b;
}

inline int letter_pos(const char *s, char c) {
  for (int t = 0; t < 4; ++t)
    if (s[t] == c) return t;
  return -1;
}

inline int block_of(const char *letters, const std::map<char, int> &spin) {
  int b = 0;
  for (int t = 0; t < 4; ++t) b |= spin.at(letters[t]) << (3 - t);
  return b;
}

// One permutation of a source block into GEMM operand layout:
// buf[(x0 r + x1) ld + x2 r + x3] = src_block[sum_t x_t st[t]].
struct PermOp {
  int src, block;  // source tensor, canonical block
  int layout;      // index into Plan::layouts
  int buf;         // operand buffer id
};

struct GemmOp {
  int a_buf, b_buf;   // operand buffer ids
  int out, block;     // output tensor and canonical block
  int stage;
  int accumulate;     // 0 for the first term of an output block
  int term;           // term index within the output block
  double alpha;       // 2 where the term stands for itself and its pair-exchanged twin
};

// K letters that are the two indices of one pair (positions 0,1 or 2,3) of a
// source tensor: the source is antisymmetric under their exchange.
inline bool source_pair(const char *nat, const char *k) {
  const int a = letter_pos(nat, k[0]), b = letter_pos(nat, k[1]);
  return a >= 0 && b >= 0 && (a >> 1) == (b >> 1);
}

struct Plan {
  std::vector<std::string> layouts;      // source letters + row/K letters, per PermOp
  std::vector<int64_t> layout_strides;   // 4 per layout, in units of natural strides (0..3 = r^3..1)
  std::vector<PermOp> perms;
  std::vector<GemmOp> gemms;
  int num_bufs = 0;                      // operand buffers (permuted sources + intermediates)
  std::map<std::pair<int, int>, int> inter_buf;   // (tensor, canonical block) -> buffer
  std::map<std::pair<int, int>, int> product_nat; // (product tensor, canonical block) -> natural array id
  int num_nat = 0;
};

// Builds the plan (independent of r).
inline Plan build_plan() {
  Plan P;
  int ns = 0;
  const Stage *st = stages(&ns);
  // forward: the canonical output blocks each stage can produce, with their terms
  std::set<std::pair<int, int>> produced;
  auto nonzero = [&](int t, int b) {
    if (is_source(t)) return source_nonzero(b);
    return produced.count({t, canon(b)}) > 0;
  };
  std::vector<std::map<int, std::vector<std::pair<int, int>>>> terms(ns);
  std::vector<std::map<int, std::vector<double>>> alphas(ns);
  std::vector<bool> twin_pairs(ns);
  for (int s = 0; s < ns; ++s) {
    const Stage &S = st[s];
    twin_pairs[s] = is_source(S.a) && is_source(S.b) && source_pair(S.la, S.ka) && source_pair(S.lb, S.kb);
    std::string letters;
    for (const char *q : {S.la, S.lb})
      for (int t = 0; t < 4; ++t)
        if (letters.find(q[t]) == std::string::npos) letters.push_back(q[t]);
    const int nl = (int)letters.size();
    for (int m = 0; m < (1 << nl); ++m) {
      std::map<char, int> spin;
      for (int t = 0; t < nl; ++t) spin[letters[t]] = (m >> t) & 1;
      const int ba = block_of(S.la, spin), bb = block_of(S.lb, spin), bo = block_of(S.lo, spin);
      if (bo & 8) continue;  // canonical outputs only
      if (!nonzero(S.a, ba) || !nonzero(S.b, bb)) continue;
      // Where the summed index pair is one antisymmetric pair of both
      // (source) operands, the terms with its two spins exchanged are equal:
      // keep the one with the first K index alpha, counted twice.
      double alpha = 1.0;
      if (twin_pairs[s] && spin.at(S.ka[0]) != spin.at(S.ka[1])) {
        if (spin.at(S.ka[0]) == 1) continue;
        alpha = 2.0;
      }
      terms[s][bo].push_back({ba, bb});
      alphas[s][bo].push_back(alpha);
    }
    for (auto &kv : terms[s]) produced.insert({S.out, kv.first});
  }
  // backward: keep what the combination (and the trace Y) needs
  std::set<std::pair<int, int>> needed;
  int npb = 0;
  const int *pb = product_blocks(&npb);
  for (int t : {T_IL, T_IR, T_PR})
    for (int q = 0; q < npb; ++q) needed.insert({t, pb[q]});
  needed.insert({T_W, 0});  // Y[k,a] = sum_p W[p,k,p,a]: blocks (s s' s s') of "ikpa" with s' alpha
  needed.insert({T_W, 5});
  for (int s = ns - 1; s >= 0; --s) {
    const Stage &S = st[s];
    for (auto &kv : terms[s]) {
      if (!needed.count({S.out, kv.first})) continue;
      for (auto &ab : kv.second) {
        if (!is_source(S.a)) needed.insert({S.a, canon(ab.first)});
        if (!is_source(S.b)) needed.insert({S.b, canon(ab.second)});
      }
    }
  }
  // buffers and operations
  std::map<std::tuple<int, int, std::string>, int> perm_buf;
  auto layout_id = [&](int src, const char *nat, const char *rows, const char *k) {
    std::string key = std::string(nat) + ":" + rows + k;
    for (size_t q = 0; q < P.layouts.size(); ++q)
      if (P.layouts[q] == key) return (int)q;
    P.layouts.push_back(key);
    for (int t = 0; t < 4; ++t) {
      const char c = t < 2 ? rows[t] : k[t - 2];
      P.layout_strides.push_back(letter_pos(nat, c));
    }
    (void)src;
    return (int)P.layouts.size() - 1;
  };
  auto operand = [&](int tensor, int block, const char *nat, const char *rows, const char *k) {
    const int cb = canon(block);
    if (!is_source(tensor)) return P.inter_buf.at({tensor, cb});
    const int lay = layout_id(tensor, nat, rows, k);
    auto key = std::make_tuple(tensor, cb, P.layouts[lay]);
    auto it = perm_buf.find(key);
    if (it != perm_buf.end()) return it->second;
    const int id = P.num_bufs++;
    perm_buf[key] = id;
    P.perms.push_back({tensor, cb, lay, id});
    return id;
  };
  for (int s = 0; s < ns; ++s) {
    const Stage &S = st[s];
    for (auto &kv : terms[s]) {
      const int bo = kv.first;
      if (!needed.count({S.out, bo})) continue;
      if (is_product(S.out)) {
        P.product_nat[{S.out, bo}] = P.num_nat++;
      } else {
        P.inter_buf[{S.out, bo}] = P.num_bufs++;
      }
      int term = 0;
      const std::vector<double> &al = alphas[s][bo];
      for (auto &ab : kv.second) {
        GemmOp g{};
        g.alpha = al[term];
        g.a_buf = operand(S.a, ab.first, S.la, S.ra, S.ka);
        g.b_buf = operand(S.b, ab.second, S.lb, S.rb, S.kb);
        g.out = S.out;
        g.block = bo;
        g.stage = s;
        g.accumulate = term > 0;
        g.term = term++;
        P.gemms.push_back(g);
      }
    }
  }
  return P;
}

// Output strides of stage s for row letters (m1, m0) and column letters
// (n1, n0), in elements, for orbital count r and operand row stride ld.
inline void gemm_out_strides(const Stage &S, int64_t r, int64_t ld, int64_t out[4]) {
  int64_t w[4];
  if (is_product(S.out)) {
    w[0] = r * r * r; w[1] = r * r; w[2] = r; w[3] = 1;
  } else {
    w[0] = r * ld; w[1] = ld; w[2] = r; w[3] = 1;
  }
  const char lt[4] = {S.ra[0], S.ra[1], S.rb[0], S.rb[1]};
  for (int t = 0; t < 4; ++t) out[t] = w[letter_pos(S.lo, lt[t])];
}

}  // namespace ny
}  // namespace acse
