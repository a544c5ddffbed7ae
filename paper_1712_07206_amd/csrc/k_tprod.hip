// Per-atom T products  Y_a = T_t(a) [A_a; B_a]  (the hoisted L-sum of Eq. 5;
// the paper evaluates the same products as the per-atom zgemm/zhemm loops of
// Alg. 3).  One complex GEMM per atom, M = K = 2N_L, N = padded N_G, on FP64
// MFMA (v_mfma_f64_16x16x4f64, four real products per complex one).
//
// Workgroup: 256 threads = 4 waves, output tile 64 rows x 64 columns, each
// wave 32 x 32 (2 x 2 MFMA blocks).  T is staged transposed in LDS so the
// A-operand fragment (16 rows at one k) is a contiguous LDS read.
#include "hs_internal.h"

namespace hsb {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 16;

__device__ inline int atom_type_of(const CellArgs& c, int atom) {
  int t = 0;
  while (t + 1 < c.n_types && atom >= c.type_start[t + 1]) ++t;
  return t;
}

__global__ void __launch_bounds__(256) k_tprod(CellArgs c, const double2* __restrict__ T, const double2* __restrict__ W,
                                               double2* __restrict__ Y, int n_pad) {
  __shared__ double2 sT[TK][TM + 1];
  __shared__ double2 sW[TK][TN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int col0 = blockIdx.x * TN;
  const int r0 = blockIdx.y * TM;
  const int atom = blockIdx.z;
  const int M = 2 * c.n_l;
  const double2* Tt = T + (int64_t)atom_type_of(c, atom) * M * M;
  const double2* Wa = W + (int64_t)atom * M * n_pad;
  double2* Ya = Y + (int64_t)atom * M * n_pad;

  d4 yr[2][2], yi[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      yr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      yi[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  for (int kc = 0; kc < M; kc += TK) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 256 * i;
      const int r = e >> 4, k = e & 15;
      double2 v = make_double2(0.0, 0.0);
      if (r0 + r < M && kc + k < M) v = Tt[(int64_t)(r0 + r) * M + kc + k];
      sT[k][r] = v;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 256 * i;
      const int k = e >> 6, cc = e & 63;
      double2 v = make_double2(0.0, 0.0);
      if (kc + k < M) v = Wa[(int64_t)(kc + k) * n_pad + col0 + cc];
      sW[k][cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double tr[2], ti[2], tn[2], wre[2], wim[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const double2 a = sT[kk][wr * 32 + i * 16 + (lane & 15)];
        tr[i] = a.x; ti[i] = a.y; tn[i] = -a.y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double2 b = sW[kk][wc * 32 + j * 16 + (lane & 15)];
        wre[j] = b.x; wim[j] = b.y;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) yr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(tr[i], wre[j], yr[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) yi[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(tr[i], wim[j], yi[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) yr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(tn[i], wim[j], yr[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) yi[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ti[i], wre[j], yi[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // D layout of the 16x16 f64 MFMA: lane l, element q -> row l/16 + 4q, column l%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + wr * 32 + i * 16 + (lane >> 4) + 4 * q;
        const int col = col0 + wc * 32 + j * 16 + (lane & 15);
        if (r < M) Ya[(int64_t)r * n_pad + col] = make_double2(yr[i][j][q], yi[i][j][q]);
      }
}

}  // namespace

hipError_t launch_tprod(const CellArgs& c, const double2* T, const double2* W, double2* Y, int n_pad,
                        hipStream_t s) {
  const int M = 2 * c.n_l;
  dim3 grid(n_pad / TN, (M + TM - 1) / TM, c.n_atoms);
  hipLaunchKernelGGL(k_tprod, grid, dim3(256), 0, s, c, T, W, Y, n_pad);
  return hipGetLastError();
}

}  // namespace hsb
