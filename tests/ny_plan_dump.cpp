#include <cstdio>
// Prints the Nakatsuji-Yasuda spin-block plan (host logic of the library,
// paper_2604_02550_amd/csrc/ny_plan.h) as JSON, for tests/test_ny_plan.py.
#include "ny_plan.h"
using namespace acse::ny;
int main() {
  Plan P = build_plan();
  int ns; const Stage *st = stages(&ns);
  printf("{\"layouts\": [");
  for (size_t q = 0; q < P.layouts.size(); ++q) printf("%s[%lld,%lld,%lld,%lld]", q ? "," : "",
      (long long)P.layout_strides[4*q], (long long)P.layout_strides[4*q+1], (long long)P.layout_strides[4*q+2], (long long)P.layout_strides[4*q+3]);
  printf("], \"operands\": [");
  for (size_t q = 0; q < P.operands.size(); ++q) { auto &o = P.operands[q]; printf("%s[%d,%d,%d,%d,%g,%d,%d,%d,%d]", q ? "," : "", o.t1, o.b1, o.t2, o.b2, o.c2, o.layout, o.phase, o.buf, o.packed); }
  printf("], \"products\": [");
  for (size_t q = 0; q < P.products.size(); ++q) { auto &g = P.products[q]; printf("%s[%d,%d,%d,%d,%d,%d,%d,%d,%g,%d]", q ? "," : "", g.a_buf, g.b_buf, g.out, g.block, g.stage, g.phase, g.accumulate, g.term, g.alpha, g.packed); }
  printf("], \"unscrambles\": [");
  for (size_t q = 0; q < P.unscrambles.size(); ++q) { auto &u = P.unscrambles[q]; printf("%s[%d,%d,%d,%d]", q ? "," : "", u.out, u.bx, u.by, u.phase); }
  printf("], \"staging\": [");
  bool first = true;
  for (auto &kv : P.staging) { printf("%s[%d,%d,%d]", first ? "" : ",", kv.first.first, kv.first.second, kv.second); first = false; }
  printf("], \"prod\": [");
  first = true;
  for (auto &kv : P.product_nat) { printf("%s[%d,%d,%d]", first ? "" : ",", kv.first.first, kv.first.second, kv.second); first = false; }
  printf("], \"nbufs\": %d, \"stages\": [", P.num_bufs);
  for (int s = 0; s < ns; ++s) printf("%s[\"%s\",\"%s\",\"%s\",\"%s\",\"%s\"]", s ? "," : "", st[s].la, st[s].ra, st[s].lb, st[s].rb, st[s].lo);
  printf("]}\n");
}
