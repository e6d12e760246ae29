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
// them), counts the two equal opposite-spin terms of a summed antisymmetric
// pair once with weight 2, and computes two output blocks that share their
// operands crosswise (x = A1 B1 + A2 B2, y = A1 B2 + A2 B1) from the products
// of the sums and of the differences.  It emits the operand builds (source
// blocks permuted into GEMM operand layout, intermediates converted from
// their FP64 staging, and the sums and differences), the product list and the
// unscrambling passes: 18 block products per map.
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

// K letters that are the two indices of one pair (positions 0,1 or 2,3) of a
// source tensor: the source is antisymmetric under their exchange.
inline bool source_pair(const char *nat, const char *k) {
  const int a = letter_pos(nat, k[0]), b = letter_pos(nat, k[1]);
  return a >= 0 && b >= 0 && (a >> 1) == (b >> 1);
}

// One GEMM operand built in operand layout: T1[b1] + c2 T2[b2] (t2 < 0: T1[b1]
// alone), canonical blocks of one tensor kind.  Sources are permuted from
// their natural arrays (layout >= 0); intermediates are read from their FP64
// staging buffers in the same layout (layout < 0).
struct OperandBuild {
  int t1, b1, t2, b2;
  double c2;
  int layout;
  int phase;   // 0: read by the first-stage products, 1: by the second stages
  int buf;     // operand buffer id
  int packed;  // K over the pairs k0 < k1 only (rows all r^2): see Product::packed
};

struct Product {
  int a_buf, b_buf;  // operand buffer ids
  int out, block;    // output tensor and canonical block
  int stage, phase;
  int accumulate;    // 0 for the first term of an output block
  int term;          // term index within the output block
  double alpha;      // 2 where the term stands for itself and its pair-exchanged twin
  int packed;        // the summed pair is antisymmetric within both operand blocks (equal
                     // spins): K runs over k0 < k1 only, alpha doubled
};

// Two output blocks x, y with x = A1 B1 + A2 B2 and y = A1 B2 + A2 B1 are
// computed as P = (A1 + A2)(B1 + B2) into x and Q = (A1 - A2)(B1 - B2) into y,
// then (x, y) <- ((x + y) / 2, (x - y) / 2): two products instead of four.
struct Unscramble {
  int out, bx, by;
  int phase;
};

struct Plan {
  std::vector<std::string> layouts;      // source letters + row/K letters
  std::vector<int64_t> layout_strides;   // 4 per layout, in units of natural strides (0..3 = r^3..1)
  std::vector<OperandBuild> operands;
  std::vector<Product> products;
  std::vector<Unscramble> unscrambles;
  int num_bufs = 0;                                // operand buffers
  std::map<std::pair<int, int>, int> staging;      // (intermediate, canonical block) -> FP64 staging buffer
  std::map<std::pair<int, int>, int> product_nat;  // (product tensor, canonical block) -> natural array id
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
  std::vector<std::map<int, std::vector<int>>> packs(ns);
  for (int s = 0; s < ns; ++s) {
    const Stage &S = st[s];
    const bool twin_pairs =
        is_source(S.a) && is_source(S.b) && source_pair(S.la, S.ka) && source_pair(S.lb, S.kb);
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
      // With equal spins the pair is antisymmetric within both blocks: the
      // sum over k0 != k1 is twice the sum over k0 < k1.
      double alpha = 1.0;
      int packed = 0;
      if (twin_pairs && spin.at(S.ka[0]) != spin.at(S.ka[1])) {
        if (spin.at(S.ka[0]) == 1) continue;
        alpha = 2.0;
      } else if (twin_pairs) {
        alpha = 2.0;
        packed = 1;
      }
      terms[s][bo].push_back({canon(ba), canon(bb)});
      alphas[s][bo].push_back(alpha);
      packs[s][bo].push_back(packed);
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
        if (!is_source(S.a)) needed.insert({S.a, ab.first});
        if (!is_source(S.b)) needed.insert({S.b, ab.second});
      }
    }
  }
  // output storage
  for (int s = 0; s < ns; ++s)
    for (auto &kv : terms[s]) {
      if (!needed.count({st[s].out, kv.first})) continue;
      if (is_product(st[s].out)) P.product_nat[{st[s].out, kv.first}] = P.num_nat++;
      else P.staging[{st[s].out, kv.first}] = (int)P.staging.size();
    }
  // operands, shared by key
  std::map<std::tuple<std::string, int, int, int, int, double, int>, int> op_buf;
  auto layout_id = [&](const char *nat, const char *rows, const char *k) {
    std::string key = std::string(nat) + ":" + rows + k;
    for (size_t q = 0; q < P.layouts.size(); ++q)
      if (P.layouts[q] == key) return (int)q;
    P.layouts.push_back(key);
    for (int t = 0; t < 4; ++t) {
      const char c = t < 2 ? rows[t] : k[t - 2];
      P.layout_strides.push_back(letter_pos(nat, c));
    }
    return (int)P.layouts.size() - 1;
  };
  auto operand = [&](int s, int side, int t, int b1, int b2, double c2, int packed) {
    const Stage &S = st[s];
    const int lay = is_source(t) ? (side ? layout_id(S.lb, S.rb, S.kb) : layout_id(S.la, S.ra, S.ka)) : -1;
    const std::string lk = lay >= 0 ? P.layouts[lay] : std::string("staging");
    auto key = std::make_tuple(lk, t, b1, b2 < 0 ? -1 : t, b2, c2, packed);
    auto it = op_buf.find(key);
    if (it != op_buf.end()) return it->second;
    const int id = P.num_bufs++;
    op_buf[key] = id;
    P.operands.push_back({t, b1, b2 < 0 ? -1 : t, b2, c2, lay, s >= ns / 2 ? 1 : 0, id, packed});
    return id;
  };
  for (int s = 0; s < ns; ++s) {
    const Stage &S = st[s];
    const int phase = s >= ns / 2 ? 1 : 0;
    std::set<int> done;
    // crosswise pairs of output blocks
    for (auto &x : terms[s]) {
      if (!needed.count({S.out, x.first}) || done.count(x.first) || x.second.size() != 2) continue;
      const auto &tx = x.second;
      if (alphas[s][x.first][0] != 1.0 || alphas[s][x.first][1] != 1.0 || packs[s][x.first][0] ||
          packs[s][x.first][1])
        continue;
      const int a1 = tx[0].first, b1 = tx[0].second, a2 = tx[1].first, b2 = tx[1].second;
      if (a1 == a2 || b1 == b2) continue;
      for (auto &y : terms[s]) {
        if (y.first == x.first || !needed.count({S.out, y.first}) || done.count(y.first) || y.second.size() != 2)
          continue;
        if (alphas[s][y.first][0] != 1.0 || alphas[s][y.first][1] != 1.0 || packs[s][y.first][0] ||
            packs[s][y.first][1])
          continue;
        std::set<std::pair<int, int>> want = {{a1, b2}, {a2, b1}}, have(y.second.begin(), y.second.end());
        if (want != have) continue;
        const int ap = operand(s, 0, S.a, a1, a2, 1.0, 0), bp = operand(s, 1, S.b, b1, b2, 1.0, 0);
        const int am = operand(s, 0, S.a, a1, a2, -1.0, 0), bm = operand(s, 1, S.b, b1, b2, -1.0, 0);
        P.products.push_back({ap, bp, S.out, x.first, s, phase, 0, 0, 1.0, 0});
        P.products.push_back({am, bm, S.out, y.first, s, phase, 0, 0, 1.0, 0});
        P.unscrambles.push_back({S.out, x.first, y.first, phase});
        done.insert(x.first);
        done.insert(y.first);
        break;
      }
    }
    for (auto &x : terms[s]) {
      if (!needed.count({S.out, x.first}) || done.count(x.first)) continue;
      int term = 0;
      for (size_t q = 0; q < x.second.size(); ++q) {
        const int pk = packs[s][x.first][q];
        const int ab = operand(s, 0, S.a, x.second[q].first, -1, 0.0, pk);
        const int bb = operand(s, 1, S.b, x.second[q].second, -1, 0.0, pk);
        P.products.push_back({ab, bb, S.out, x.first, s, phase, term > 0, term, alphas[s][x.first][q], pk});
        ++term;
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
