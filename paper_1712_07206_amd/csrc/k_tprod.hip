// Per-atom T products  Y_a = T_t(a) [A_a; B_a]  (the hoisted L-sum of Eq. 5;
// the paper evaluates the same products as the per-atom zgemm/zhemm loops of
// Alg. 3).  One complex GEMM per atom, M = K = 2N_L, N = padded N_G.
//
// The products run on the contraction's 3M tile routine (k_tprod3m in k_hs.hip,
// three real FP64 MFMAs per complex multiply-add).  Its left operand is staged
// by straight copies of rows, so T is first laid out here transposed and
// zero-padded per type: TT[t][k][r] = T[t][r][k] for r, k < M, zero up to
// [round16(M)][round128(M)].  The padding makes the rows of a 16-row chunk past
// M (which belong to the next atom, or to the zero rows past K) contribute
// nothing, and the tile rows past M compute zeros that are not stored.
#include "hs_internal.h"

namespace hsb {

namespace {

__global__ void __launch_bounds__(256) k_tpad(const double2* __restrict__ T, int M, int Kc, int MP,
                                              double2* __restrict__ TT) {
  const int r = blockIdx.x * 256 + threadIdx.x, k = blockIdx.y, t = blockIdx.z;
  if (r >= MP) return;
  double2 v = make_double2(0.0, 0.0);
  if (r < M && k < M) v = T[((int64_t)t * M + r) * M + k];
  TT[((int64_t)t * Kc + k) * MP + r] = v;
}

}  // namespace

hipError_t launch_tpad(const double2* T, int n_types, int M, double2* TT, hipStream_t s) {
  const int Kc = tprod_kc(M), MP = tprod_mp(M);
  hipLaunchKernelGGL(k_tpad, dim3((MP + 255) / 256, Kc, n_types), dim3(256), 0, s, T, M, Kc, MP, TT);
  return hipGetLastError();
}

hipError_t launch_tprod(const CellArgs& c, const double2* TT, const double2* W, double2* Y, int n_pad,
                        hipStream_t s) {
  return launch_tprod3m(c, TT, W, Y, n_pad, s);
}

}  // namespace hsb
