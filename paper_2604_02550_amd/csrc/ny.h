// Kernels of the Nakatsuji-Yasuda share of the residual map (ny.hip); the
// plan they execute is in ny_plan.h.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace acse {

// Canonical spin blocks of the 2-cumulant (Eq. (7)) and of X, natural r^4:
//   Daa = d2aa - 1/2 (g_pr g_qs - g_ps g_qr),  Dab = d2ab - 1/2 g_pr g_qs,
//   Dabx[p,q,r,s] = -Dab[p,q,s,r],  SD* = sigma_r D* (third index scaled),
//   Xabx[p,q,r,s] = -Xab[p,q,s,r].  With keep_d only Xabx is written (the
// cumulant blocks stand from a previous call on the same 2-RDM).
hipError_t launch_ny_sources(int r, const double *g, const double *d2aa, const double *d2ab,
                             const double *Xab, const double *sigma, double *const src[7], bool keep_d,
                             hipStream_t s);
// (x, y) <- ((x + y) / 2, (x - y) / 2) over n elements: the two blocks of a
// crosswise pair from the products of the sums and of the differences.
hipError_t launch_ny_unscramble(int64_t n, double *x, double *y, hipStream_t s);
// Y[k,a] = sum_p (W0 + W5)[(p r + k) ld + p r + a] (the alpha-alpha block of
// the partial trace of the first intermediate of T_il).
hipError_t launch_ny_trace_y(int r, int64_t ld, const double *W0, const double *W5, double *Y, hipStream_t s);
// S_aa -= C_aa, S_ab -= C_ab with C = B - B(k<->l) and
// B = 4 [sw(T_il) + T_pl - 2 sw(T_ir) - 2 T_pr] on the canonical blocks
// 0000, 0101, 0110 (slots 0, 1, 2); T_pl = sum_a Y[k,a] SD[i,j,a,l].
// Two passes, one block per (i,j) slab each: the B blocks into B[0..2] (the
// i <-> j exchange reads whole (k,l) slabs; Y and the SD slab in LDS), then
// the k <-> l exchange through slabs in LDS.  Each needs 2 r (r+1) doubles of
// LDS (r <= 96: 149 KB).
struct NyCombineArgs {
  const double *il[3], *ir[3], *pr[3], *sd[3];
  const double *Y;
  double *B[3];
  double *Saa, *Sab;
};
hipError_t launch_ny_combine(int r, const NyCombineArgs &a, hipStream_t s);

}  // namespace acse
