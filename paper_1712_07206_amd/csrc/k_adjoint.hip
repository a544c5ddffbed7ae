// Adjoint of the H/S build for a real loss L(H, S) with Hermitian incoming
// gradients gH = dL/dRe H + i dL/dIm H and gS (likewise).
//
// With W the stacked coefficients (rows k = (atom, A|B, L)), Y_a = T_t W_a and
// P_H = W gH, P_S = W gS (both [K][N_G]):
//   grad T_t   = sum_{a in t} P_H,a W_a^H                          (2N_L x 2N_L per type)
//   grad tau_a = -2 sum_G K_G Im c_a(G),
//   c_a(G)     = sum_{k in a} conj(P_H[k][G]) Y[k][G] + conj(P_S[k][G]) lam_k W[k][G]
// since every coefficient of atom a carries the phase e^{iK_G.tau_a}
// (A and B of Eq. 2) and H, S are the sums of Eqs. 4-5.  Nothing is kept
// from the forward: W and Y are rebuilt by the same kernels.
//
//   k_transpose,   W^T and zero-padded gH, gS for the products P_H and P_S, which
//   k_pad_square   run in the 3M form in k_pgemm3m (with the forward's tile routine)
//   k_gradT        per-atom partials P_H,a W_a^H (FP64 MFMA), one workgroup per
//                  (64 x 64 tile, atom); k_gradT_reduce sums the atoms of a type
//                  in a fixed order (deterministic)
//   k_gradtau      per (atom, 256-column block) partial sums; k_gradtau_reduce
//                  adds the blocks in a fixed order
#include "hs_internal.h"

namespace hsb {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

#define MFMA(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

// ---- grad T partials: part[atom][r][c] = sum_G P_H[a*M + r][G] conj(W[a*M + c][G]) ---------
constexpr int TT = 64, TKG = 16;

__global__ void __launch_bounds__(256) k_gradT(const d2* __restrict__ P, const d2* __restrict__ W, int M, int n_pad,
                                               d2* __restrict__ part) {
  __shared__ d2 sP[TKG][TT + 1];
  __shared__ d2 sW[TKG][TT + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int ntile = (M + TT - 1) / TT;
  const int r0 = (blockIdx.x / ntile) * TT, c0 = (blockIdx.x % ntile) * TT;
  const int atom = blockIdx.y;
  const d2* Pa = P + (int64_t)atom * M * n_pad;
  const d2* Wa = W + (int64_t)atom * M * n_pad;
  d4 gr[2][2], gi[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      gr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      gi[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  for (int kc = 0; kc < n_pad; kc += TKG) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 256 * i;
      const int g = e & 15, r = e >> 4;
      d2 vp = d2{0.0, 0.0}, vw = d2{0.0, 0.0};
      if (r0 + r < M) vp = Pa[(int64_t)(r0 + r) * n_pad + kc + g];
      if (c0 + r < M) vw = Wa[(int64_t)(c0 + r) * n_pad + kc + g];
      sP[g][r] = vp;
      sW[g][r] = vw;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < TKG / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double pr[2], pi[2], wre[2], wim[2], wneg[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const d2 a = sP[kk][wr * 32 + i * 16 + (lane & 15)];
        pr[i] = a.x; pi[i] = a.y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const d2 b = sW[kk][wc * 32 + j * 16 + (lane & 15)];
        wre[j] = b.x; wim[j] = b.y; wneg[j] = -b.y;
      }
      // P conj(W): re = pr wr + pi wi, im = pi wr - pr wi
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) gr[i][j] = MFMA(pr[i], wre[j], gr[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) gi[i][j] = MFMA(pi[i], wre[j], gi[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) gr[i][j] = MFMA(pi[i], wim[j], gr[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) gi[i][j] = MFMA(pr[i], wneg[j], gi[i][j]);
    }
    __syncthreads();
  }
  d2* out = part + (int64_t)atom * M * M;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + wr * 32 + i * 16 + (lane >> 4) + 4 * q;
        const int c = c0 + wc * 32 + j * 16 + (lane & 15);
        if (r < M && c < M) out[(int64_t)r * M + c] = d2{gr[i][j][q], gi[i][j][q]};
      }
}

__global__ void __launch_bounds__(256) k_gradT_reduce(CellArgs c, const d2* __restrict__ part, int M,
                                                      d2* __restrict__ gT) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (idx >= (int64_t)M * M) return;
  d2 acc = d2{0.0, 0.0};
  for (int a = c.type_start[t]; a < c.type_start[t + 1]; ++a) acc += part[(int64_t)a * M * M + idx];
  gT[(int64_t)t * M * M + idx] = acc;
}

// ---- grad tau --------------------------------------------------------------------------
constexpr int TB = 256;

__global__ void __launch_bounds__(TB) k_gradtau(const d2* __restrict__ PH, const d2* __restrict__ PS,
                                                const d2* __restrict__ Y, const d2* __restrict__ W,
                                                const double* __restrict__ lam, const double* __restrict__ kv,
                                                int M, int n, int n_pad, double* __restrict__ part) {
  __shared__ double red[3][TB / 64];
  const int G = blockIdx.x * TB + threadIdx.x;
  const int atom = blockIdx.y;
  double s = 0.0;
  if (G < n) {
    const int64_t base = (int64_t)atom * M * n_pad + G;
    for (int r = 0; r < M; ++r) {
      const int64_t o = base + (int64_t)r * n_pad;
      const d2 ph = PH[o], y = Y[o], ps = PS[o], w = W[o];
      const double l = lam[atom * M + r];
      // Im(conj(ph) y) + l Im(conj(ps) w)
      s += ph.x * y.y - ph.y * y.x + l * (ps.x * w.y - ps.y * w.x);
    }
  }
  double v[3] = {0.0, 0.0, 0.0};
  if (G < n) {
    v[0] = s * kv[4 * (int64_t)G + 0];
    v[1] = s * kv[4 * (int64_t)G + 1];
    v[2] = s * kv[4 * (int64_t)G + 2];
  }
  // wave reduction (fixed butterfly order), then across the block's waves
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[d] += __shfl_xor(v[d], off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    red[0][wave] = v[0];
    red[1][wave] = v[1];
    red[2][wave] = v[2];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double acc = 0.0;
    for (int w = 0; w < TB / 64; ++w) acc += red[threadIdx.x][w];
    part[((int64_t)atom * gridDim.x + blockIdx.x) * 3 + threadIdx.x] = acc;
  }
}

__global__ void __launch_bounds__(64) k_gradtau_reduce(const double* __restrict__ part, int nblocks, int n_atoms,
                                                       double* __restrict__ gtau) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n_atoms) return;
  const int atom = i / 3, d = i % 3;
  double acc = 0.0;
  for (int b = 0; b < nblocks; ++b) acc += part[((int64_t)atom * nblocks + b) * 3 + d];
  gtau[i] = -2.0 * acc;
}

// ---- operand preparation for the 3M products --------------------------------------
// WT[G][k] = W[k][G] for k < K_pad, 0 for K_pad <= k < Kt; 32 x 32 tiles through LDS.
__global__ void __launch_bounds__(256) k_transpose(const d2* __restrict__ W, int K_pad, int n_pad, int Kt,
                                                   d2* __restrict__ WT) {
  __shared__ d2 t[32][33];
  const int k0 = blockIdx.x * 32, g0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r;
    t[r][tx] = k < K_pad ? W[(int64_t)k * n_pad + g0 + tx] : d2{0.0, 0.0};
  }
  __syncthreads();
#pragma unroll
  for (int r = ty; r < 32; r += 8) WT[(int64_t)(g0 + r) * Kt + k0 + tx] = t[tx][r];
}

// gp[r][c] = g[r][c] for r, c < n, 0 elsewhere (r, c < n_pad).
__global__ void __launch_bounds__(256) k_pad_square(const d2* __restrict__ g, int n, int n_pad, d2* __restrict__ gp) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n_pad) return;
  for (int r = blockIdx.y; r < n_pad; r += gridDim.y)
    gp[(int64_t)r * n_pad + c] = (r < n && c < n) ? g[(int64_t)r * n + c] : d2{0.0, 0.0};
}

}  // namespace

int gradtau_blocks(int n) { return (n + TB - 1) / TB; }

hipError_t launch_transpose(const double2* W, int K_pad, int n_pad, int Kt, double2* WT, hipStream_t s) {
  if (Kt % 32 || n_pad % 32 || Kt < K_pad) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_transpose, dim3(Kt / 32, n_pad / 32), dim3(256), 0, s, (const d2*)W, K_pad, n_pad, Kt,
                     (d2*)WT);
  return hipGetLastError();
}

hipError_t launch_pad_square(const double2* g, int n, int n_pad, double2* gp, hipStream_t s) {
  hipLaunchKernelGGL(k_pad_square, dim3((n_pad + 255) / 256, n_pad < 4096 ? n_pad : 4096), dim3(256), 0, s,
                     (const d2*)g, n, n_pad, (d2*)gp);
  return hipGetLastError();
}

hipError_t launch_gradT(const CellArgs& c, const double2* PH, const double2* W, int n_pad, double2* part,
                        double2* gT, hipStream_t s) {
  const int M = 2 * c.n_l;
  const int ntile = (M + TT - 1) / TT;
  hipLaunchKernelGGL(k_gradT, dim3(ntile * ntile, c.n_atoms), dim3(256), 0, s, (const d2*)PH, (const d2*)W, M,
                     n_pad, (d2*)part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gradT_reduce, dim3((M * M + 255) / 256, c.n_types), dim3(256), 0, s, c, (const d2*)part, M,
                     (d2*)gT);
  return hipGetLastError();
}

hipError_t launch_gradtau(const CellArgs& c, const double2* PH, const double2* PS, const double2* Y,
                          const double2* W, const double* lam, const double* kv, int n, int n_pad, double* part,
                          double* gtau, hipStream_t s) {
  const int M = 2 * c.n_l;
  const int nb = gradtau_blocks(n);
  hipLaunchKernelGGL(k_gradtau, dim3(nb, c.n_atoms), dim3(TB), 0, s, (const d2*)PH, (const d2*)PS, (const d2*)Y,
                     (const d2*)W, lam, kv, M, n, n_pad, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gradtau_reduce, dim3((3 * c.n_atoms + 63) / 64), dim3(64), 0, s, (const double*)part, nb,
                     c.n_atoms, gtau);
  return hipGetLastError();
}

}  // namespace hsb
