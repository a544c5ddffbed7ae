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
//   k_pgemm        P_H and P_S in one pass (shared left operand W), FP64 MFMA,
//                  8 waves, double-buffered LDS
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

// ---- P_H = W gH, P_S = W gS -------------------------------------------------------------
// Tile 128 (k) x 64 (G) for both outputs; 8 waves of 32 x 32 (two per SIMD).  The
// contraction runs over G' in chunks of 16 through double-buffered LDS with a
// register prefetch of the next chunk.  W is staged transposed (sA[G'][k], padded
// row) so the A fragment (16 k rows at one G') is a contiguous LDS read.
constexpr int PM = 128, PN = 64, PK = 16, PT = 512;

__global__ void __launch_bounds__(PT, 1) k_pgemm(const d2* __restrict__ W, const d2* __restrict__ gH,
                                                 const d2* __restrict__ gS, int K_pad, int n, int n_pad,
                                                 d2* __restrict__ PH, d2* __restrict__ PS) {
  __shared__ d2 sA[2][PK][PM + 1];
  __shared__ d2 sH[2][PK][PN];
  __shared__ d2 sS[2][PK][PN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;  // rows wr*32, columns wc*32
  const int col0 = blockIdx.x * PN;
  const int row0 = blockIdx.y * PM;
  d4 hr[2][2], hi[2][2], sr[2][2], si[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      hr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      hi[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      sr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      si[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  // staging: A 16 x 128 (4 per thread, transposed on store), gH and gS 16 x 64 (2 each)
  d2 pa[4], ph[2], ps[2];
#define PG_LOAD(kc)                                                                   \
  do {                                                                                \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                   \
      const int e = tid + PT * i;                                                     \
      const int c = e & 15, r = e >> 4;                                               \
      pa[i] = row0 + r < K_pad ? W[(int64_t)(row0 + r) * n_pad + (kc) + c] : d2{0.0, 0.0}; \
    }                                                                                 \
    _Pragma("unroll") for (int i = 0; i < 2; ++i) {                                   \
      const int e = tid + PT * i;                                                     \
      const int r = e >> 6, c = e & 63;                                               \
      const int gp = (kc) + r, gc = col0 + c;                                         \
      const bool ok = gp < n && gc < n;                                               \
      ph[i] = ok ? gH[(int64_t)gp * n + gc] : d2{0.0, 0.0};                           \
      ps[i] = ok ? gS[(int64_t)gp * n + gc] : d2{0.0, 0.0};                           \
    }                                                                                 \
  } while (0)
#define PG_STORE(b)                                    \
  do {                                                 \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {    \
      const int e = tid + PT * i;                      \
      sA[b][e & 15][e >> 4] = pa[i];                   \
    }                                                  \
    _Pragma("unroll") for (int i = 0; i < 2; ++i) {    \
      const int e = tid + PT * i;                      \
      sH[b][e >> 6][e & 63] = ph[i];                   \
      sS[b][e >> 6][e & 63] = ps[i];                   \
    }                                                  \
  } while (0)

  const int nchunks = n_pad / PK;
  PG_LOAD(0);
  PG_STORE(0);
  __syncthreads();
  for (int ch = 0; ch < nchunks; ++ch) {
    const int b = ch & 1;
    if (ch + 1 < nchunks) PG_LOAD((ch + 1) * PK);
#pragma unroll
    for (int ks = 0; ks < PK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double ar[2], ai[2], an[2], hre[2], him[2], sre[2], sim[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const d2 a = sA[b][kk][wr * 32 + i * 16 + (lane & 15)];
        ar[i] = a.x; ai[i] = a.y; an[i] = -a.y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const d2 bh = sH[b][kk][wc * 32 + j * 16 + (lane & 15)];
        const d2 bs = sS[b][kk][wc * 32 + j * 16 + (lane & 15)];
        hre[j] = bh.x; him[j] = bh.y; sre[j] = bs.x; sim[j] = bs.y;
      }
      // (ar + i ai)(br + i bi): re = ar br - ai bi, im = ar bi + ai br
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) hr[i][j] = MFMA(ar[i], hre[j], hr[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) hi[i][j] = MFMA(ar[i], him[j], hi[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) sr[i][j] = MFMA(ar[i], sre[j], sr[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) si[i][j] = MFMA(ar[i], sim[j], si[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) hr[i][j] = MFMA(an[i], him[j], hr[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) hi[i][j] = MFMA(ai[i], hre[j], hi[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) sr[i][j] = MFMA(an[i], sim[j], sr[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) si[i][j] = MFMA(ai[i], sre[j], si[i][j]);
    }
    if (ch + 1 < nchunks) PG_STORE(b ^ 1);
    __syncthreads();
  }
#undef PG_LOAD
#undef PG_STORE
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + wr * 32 + i * 16 + (lane >> 4) + 4 * q;
        const int col = col0 + wc * 32 + j * 16 + (lane & 15);
        if (row < K_pad) {
          const int64_t o = (int64_t)row * n_pad + col;
          PH[o] = d2{hr[i][j][q], hi[i][j][q]};
          PS[o] = d2{sr[i][j][q], si[i][j][q]};
        }
      }
}

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

}  // namespace

int gradtau_blocks(int n) { return (n + TB - 1) / TB; }

hipError_t launch_pgemm(const double2* W, const double2* gH, const double2* gS, int K_pad, int n, int n_pad,
                        double2* PH, double2* PS, hipStream_t s) {
  dim3 grid(n_pad / PN, (K_pad + PM - 1) / PM);
  hipLaunchKernelGGL(k_pgemm, grid, dim3(PT), 0, s, (const d2*)W, (const d2*)gH, (const d2*)gS, K_pad, n, n_pad,
                     (d2*)PH, (d2*)PS);
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
