// Fused Hermitian contractions (Eqs. 6-7 after stacking, Sec. 3 / Fig. 1):
//
//   S[G'][G] = sum_k conj(W[k][G']) lam[k] W[k][G]     (herk, one triangle)
//   H[G'][G] = sum_k conj(W[k][G']) Y[k][G]            (herkx, one triangle)
//
// over the stacked index k = (atom, A|B, L) of width 2 N_atoms N_L.  The
// paper's refined algorithm (Alg. 3) gets H from zher2k + zherkx over the
// A and B halves separately (12 N_A N_L N_G^2 flops); with Y = T W already
// formed per atom, one herkx over the full stacked width gives the same H in
// 8 N_A N_L N_G^2, and S shares its left operand W.
//
// Complex FP64 on v_mfma_f64_16x16x4f64.  Workgroup: output tile 128 (G') x 64
// (G) for both H and S.  Two variants:
//   8 waves of 32 x 32 (two waves per SIMD, which hides the chunk barriers):
//     three real MFMAs per complex multiply-add (the 3M form, hs_tile3m below),
//     operand strips copied straight into double-buffered LDS;
//   4 waves of 64 x 32 (accumulators in AGPRs, one wave per SIMD): four real
//     MFMAs per complex multiply-add, Re += Wr^T Yr + Wi^T Yi,
//     Im += Wr^T Yi - Wi^T Yr, with a register prefetch of the next chunk.
// The two agree to FP64 rounding.  K is staged 16 rows at a time.  Only tiles
// that touch the upper triangle are computed; they are numbered over 128 x 128
// super-tiles (grouped order, tiles.h) and the numbering is dealt to the eight
// XCDs in contiguous ranges so tiles sharing a row strip share an L2.  The 3M
// tile routine also serves the per-atom T products (k_tprod3m) and the
// adjoint's products (k_pgemm3m), with the plain complex product.
//
// k_hs_fp64 computes one k-point, one workgroup per tile.  k_hs_fp64_batch is
// the persistent form for many k-points: a fixed grid (one workgroup per CU)
// walks a tile list spanning every k-point, each XCD taking one contiguous
// range of it; every tile costs the same (same stacked width), so a static
// walk balances.  Both run the same tile body, so a batched H(k) is bitwise
// equal to the single-k one.
#include <cmath>

#include "hs_internal.h"
#include "tiles.h"

namespace hsb {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int BM = 128, BN = 64, BK = 16;
#define MFMA(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

struct Smem {
  d2 L[2][BK][BM];
  d2 R[2][BK][BN];
  d2 Y[2][BK][BN];
};

// One 128 x 64 tile (rows row0.., columns col0..) of H and S, upper triangle stored.
// WR x 2 waves; each wave owns (128/WR) x 32 of both outputs: MI x 2 MFMA blocks.
// REAL: only the real parts, Re(W^H Y) and Re(W^H lam W), into double outputs (the
// real-symmetric case: half the MFMAs of the complex product).
template <int WR, bool REAL = false>
__device__ __forceinline__ void hs_tile(Smem& sm, const d2* __restrict__ W, const d2* __restrict__ Y,
                                        const double* __restrict__ lam, int K_pad, int n, int n_pad, int row0,
                                        int col0, void* __restrict__ Hv, void* __restrict__ Sv, int64_t ldh) {
  constexpr int NT = 64 * WR * 2;   // threads
  constexpr int MI = BM / WR / 16;  // row blocks per wave
  constexpr int PL = BK * BM / NT, PR = BK * BN / NT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;

  // staging map: left chunk 16 x 128 (PL per thread), right chunks 16 x 64 (PR per thread)
  d2 pl[PL], pr[PR], py[PR];
  double pm[PR];
#define HS_GLOAD(kc)                                                             \
  do {                                                                           \
    _Pragma("unroll") for (int i = 0; i < PL; ++i) {                             \
      const int e = tid + NT * i;                                                \
      pl[i] = W[(int64_t)((kc) + (e >> 7)) * n_pad + row0 + (e & 127)];          \
    }                                                                            \
    _Pragma("unroll") for (int i = 0; i < PR; ++i) {                             \
      const int e = tid + NT * i;                                                \
      const int64_t off = (int64_t)((kc) + (e >> 6)) * n_pad + col0 + (e & 63);  \
      pr[i] = W[off];                                                            \
      py[i] = Y[off];                                                            \
      pm[i] = lam[(kc) + (e >> 6)];                                              \
    }                                                                            \
  } while (0)
#define HS_LSTORE(b)                                 \
  do {                                               \
    _Pragma("unroll") for (int i = 0; i < PL; ++i) { \
      const int e = tid + NT * i;                    \
      sm.L[b][e >> 7][e & 127] = pl[i];              \
    }                                                \
    _Pragma("unroll") for (int i = 0; i < PR; ++i) { \
      const int e = tid + NT * i;                    \
      sm.R[b][e >> 6][e & 63] = pm[i] * pr[i];       \
      sm.Y[b][e >> 6][e & 63] = py[i];               \
    }                                                \
  } while (0)

  d4 hr[MI][2], hi[MI][2], sr[MI][2], si[MI][2];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      hr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      hi[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      sr[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      si[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  const int nchunks = K_pad / BK;
  HS_GLOAD(0);
  HS_LSTORE(0);
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int b = c & 1;
    if (c + 1 < nchunks) HS_GLOAD((c + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      // the next chunk goes into the other buffer mid-chunk (free since the last barrier),
      // so its LDS stores overlap the MFMAs still queued instead of delaying the barrier
      if (ks == BK / 8 && c + 1 < nchunks) HS_LSTORE(b ^ 1);
      const int kk = ks * 4 + (lane >> 4);
      double ar[MI], ai[MI], an[MI], yre[2], yim[2], wre[2], wim[2];
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const d2 a = sm.L[b][kk][wr * (BM / WR) + i * 16 + (lane & 15)];
        ar[i] = a.x; ai[i] = a.y; an[i] = -a.y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const d2 yv = sm.Y[b][kk][wc * 32 + j * 16 + (lane & 15)];
        const d2 wv = sm.R[b][kk][wc * 32 + j * 16 + (lane & 15)];
        yre[j] = yv.x; yim[j] = yv.y; wre[j] = wv.x; wim[j] = wv.y;
      }
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) hr[i][j] = MFMA(ar[i], yre[j], hr[i][j]);
      if constexpr (!REAL) {
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) hi[i][j] = MFMA(ar[i], yim[j], hi[i][j]);
      }
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) sr[i][j] = MFMA(ar[i], wre[j], sr[i][j]);
      if constexpr (!REAL) {
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) si[i][j] = MFMA(ar[i], wim[j], si[i][j]);
      }
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) hr[i][j] = MFMA(ai[i], yim[j], hr[i][j]);
      if constexpr (!REAL) {
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) hi[i][j] = MFMA(an[i], yre[j], hi[i][j]);
      }
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) sr[i][j] = MFMA(ai[i], wim[j], sr[i][j]);
      if constexpr (!REAL) {
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) si[i][j] = MFMA(an[i], wre[j], si[i][j]);
      }
    }
    __syncthreads();
  }
#undef HS_GLOAD
#undef HS_LSTORE

  // D layout of the 16x16 f64 MFMA: lane l, element q -> row l/16 + 4q, column l%16
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + wr * (BM / WR) + i * 16 + (lane >> 4) + 4 * q;
        const int col = col0 + wc * 32 + j * 16 + (lane & 15);
        if (row < n && col < n && col >= row) {
          const int64_t o = (int64_t)row * ldh + col;
          if constexpr (REAL) {
            ((double*)Hv)[o] = hr[i][j][q];
            ((double*)Sv)[o] = sr[i][j][q];
          } else {
            ((d2*)Hv)[o] = d2{hr[i][j][q], hi[i][j][q]};
            ((d2*)Sv)[o] = d2{sr[i][j][q], si[i][j][q]};
          }
        }
      }
}

// The complex contraction with three real products per complex multiply-add
// (the Gauss/3M form).  CONJ: S = sum_k conj(L) R and H = sum_k conj(L) Y, for
// Re + i Im = conj(a) b
//   P1 = a_r b_r,  P2 = a_i b_i,  P3 = (a_r - a_i)(b_r + b_i),
//   Re = P1 + P2,  Im = P3 - P1 + P2;
// otherwise the plain products S = sum_k L R, H = sum_k L Y, for a b
//   P3 = (a_r + a_i)(b_r + b_i),  Re = P1 - P2,  Im = P3 - P1 - P2.
// Each P is summed over k in its own accumulator and combined in the epilogue:
// 3 MFMAs where the plain form issues 4, for the same sums up to rounding.  The
// operand sums are formed in registers after the LDS reads.  The three K-chunk
// operands (L at the tile rows, R and Y at the tile columns: for the forward W,
// lam W prepared in HBM, and Y) are copied straight into double-buffered LDS with
// global_load_lds_dwordx4, one barrier per chunk, so no staging registers are held
// across the MFMAs.  L rows are ldL long, R and Y rows ldR; Kc (a multiple of 16)
// rows are contracted.  Stored: row < n_row, col < n_col and, with upper, col >= row.
typedef __attribute__((address_space(3))) void* lds_ptr;

template <int WR, bool CONJ>
__device__ __forceinline__ void hs_tile3m(Smem& sm, const d2* __restrict__ L, const d2* __restrict__ R,
                                          const d2* __restrict__ Y, int Kc, int ldL, int ldR, int row0, int col0,
                                          int n_row, int n_col, bool upper, d2* __restrict__ H, d2* __restrict__ S,
                                          int64_t ldh) {
  constexpr int NWV = 2 * WR;              // waves
  constexpr int MI = BM / WR / 16;         // row blocks per wave
  constexpr int NCP = BK * 2 + BK + BK;    // 1 KB copies per chunk: L rows are two copies, R and Y one
  constexpr int CPW = NCP / NWV;           // copies per wave
  constexpr int CPL = 2 * BK / NWV;        // the first CPL copies of every wave are L rows
  static_assert(NCP % NWV == 0 && (2 * BK) % NWV == 0, "copy map");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;

  // copy j: j < 2 BK: L row j/2, half j%2; then BK rows of R; then BK rows of Y
  const d2* src0[CPW];
  int dst[CPW];  // d2 offset inside one buffer of sm (L, R, Y are consecutive members)
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    const int j = wave + NWV * i;
    if (i < CPL) {
      src0[i] = L + (int64_t)(j >> 1) * ldL + row0 + (j & 1) * 64;
      dst[i] = (j >> 1) * BM + (j & 1) * 64;
    } else if (j < 3 * BK) {
      const int r = j - 2 * BK;
      src0[i] = R + (int64_t)r * ldR + col0;
      dst[i] = 2 * BK * BM + r * BN;  // after L[2][BK][BM]
    } else {
      const int r = j - 3 * BK;
      src0[i] = Y + (int64_t)r * ldR + col0;
      dst[i] = 2 * BK * BM + 2 * BK * BN + r * BN;  // after R[2][BK][BN]
    }
  }
  d2* base = &sm.L[0][0][0];
  auto issue = [&](int c, int buf) {
#pragma unroll
    for (int i = 0; i < CPW; ++i) {
      // the buffer index moves L by BK*BM and R, Y by BK*BN elements
      const int off = dst[i] + buf * (i < CPL ? BK * BM : BK * BN);
      const int64_t adv = (int64_t)c * BK * (i < CPL ? ldL : ldR);
      __builtin_amdgcn_global_load_lds((const void*)(src0[i] + adv + lane), (lds_ptr)(base + off), 16, 0, 0);
    }
  };

  d4 h1[MI][2], h2[MI][2], h3[MI][2], s1[MI][2], s2[MI][2], s3[MI][2];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      h1[i][j] = h2[i][j] = h3[i][j] = s1[i][j] = s2[i][j] = s3[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int nchunks = Kc / BK;
  issue(0, 0);
  for (int c = 0; c < nchunks; ++c) {
    const int b = c & 1;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of chunk c have landed
    __syncthreads();                // everyone's have, and buffer b^1 is free
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      // the next chunk's copies go out half-way through this one: issued right after the
      // barrier their LDS writes meet the chunk's first reads (measured: 1.8 % slower)
      if (ks == BK / 8 && c + 1 < nchunks) issue(c + 1, b ^ 1);
      const int kk = ks * 4 + (lane >> 4);
      double ar[MI], ai[MI], ad[MI], yre[2], yim[2], ys[2], wre[2], wim[2], wsum[2];
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const d2 a = sm.L[b][kk][wr * (BM / WR) + i * 16 + (lane & 15)];
        ar[i] = a.x; ai[i] = a.y; ad[i] = CONJ ? a.x - a.y : a.x + a.y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const d2 yv = sm.Y[b][kk][wc * 32 + j * 16 + (lane & 15)];
        const d2 wv = sm.R[b][kk][wc * 32 + j * 16 + (lane & 15)];
        yre[j] = yv.x; yim[j] = yv.y; ys[j] = yv.x + yv.y;
        wre[j] = wv.x; wim[j] = wv.y; wsum[j] = wv.x + wv.y;
      }
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          h1[i][j] = MFMA(ar[i], yre[j], h1[i][j]);
          s1[i][j] = MFMA(ar[i], wre[j], s1[i][j]);
        }
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          h2[i][j] = MFMA(ai[i], yim[j], h2[i][j]);
          s2[i][j] = MFMA(ai[i], wim[j], s2[i][j]);
        }
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          h3[i][j] = MFMA(ad[i], ys[j], h3[i][j]);
          s3[i][j] = MFMA(ad[i], wsum[j], s3[i][j]);
        }
    }
  }

  // D layout of the 16x16 f64 MFMA: lane l, element q -> row l/16 + 4q, column l%16
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + wr * (BM / WR) + i * 16 + (lane >> 4) + 4 * q;
        const int col = col0 + wc * 32 + j * 16 + (lane & 15);
        if (row < n_row && col < n_col && (!upper || col >= row)) {
          const int64_t o = (int64_t)row * ldh + col;
          const double p1 = h1[i][j][q], p2 = h2[i][j][q], q1 = s1[i][j][q], q2 = s2[i][j][q];
          if constexpr (CONJ) {
            H[o] = d2{p1 + p2, h3[i][j][q] - p1 + p2};
            S[o] = d2{q1 + q2, s3[i][j][q] - q1 + q2};
          } else {
            H[o] = d2{p1 - p2, h3[i][j][q] - p1 - p2};
            S[o] = d2{q1 - q2, s3[i][j][q] - q1 - q2};
          }
        }
      }
}

template <int WR, bool REAL>
__global__ void __launch_bounds__(128 * WR, 1) k_hs_fp64(const d2* __restrict__ W, const d2* __restrict__ WL,
                                                     const d2* __restrict__ Y, const double* __restrict__ lam,
                                                     int K_pad, int n, int n_pad, int nbr, int num_wg, int gr,
                                                     void* __restrict__ H, void* __restrict__ S, int64_t ldh) {
  __shared__ Smem sm;
  // dispatch is round-robin over XCDs: give XCD x the contiguous range of tile numbers
  const int x = blockIdx.x % kXcds;
  int start, len;
  xcd_range(x, num_wg, start, len);
  const int w = start + blockIdx.x / kXcds;
  int row0, col0;
  tile_origin(w, nbr, gr, row0, col0);
  if (col0 >= n) return;
  if constexpr (REAL) hs_tile<WR, true>(sm, W, Y, lam, K_pad, n, n_pad, row0, col0, H, S, ldh);
  else if constexpr (WR == 4)
    hs_tile3m<WR, true>(sm, W, WL, Y, K_pad, n_pad, n_pad, row0, col0, n, n, true, (d2*)H, (d2*)S, ldh);
  else hs_tile<WR, false>(sm, W, Y, lam, K_pad, n, n_pad, row0, col0, H, S, ldh);  // 64 x 32 per wave: plain form
}

// The 8-wave contraction with the stacked index cut into ns segments of kseg rows: workgroup
// w = (segment p, tile t), segments outermost so the tiles running together read the same
// rows; each writes its partial upper-triangle tile of H and S into Hp[p], Sp[p] ([n_pad]^2
// each).  k_sk_reduce adds the segments in order p = 0, 1, ..., so results are reproducible.
__global__ void __launch_bounds__(512, 1) k_hs_fp64_sk(const d2* __restrict__ W, const d2* __restrict__ WL,
                                                       const d2* __restrict__ Y, int K_pad, int kseg, int n,
                                                       int n_pad, int nbr, int num_wg, int total, int gr,
                                                       d2* __restrict__ Hp, d2* __restrict__ Sp) {
  __shared__ Smem sm;
  const int x = blockIdx.x % kXcds;
  int start, len;
  xcd_range(x, total, start, len);
  const int w = start + blockIdx.x / kXcds;
  const int p = w / num_wg;
  int row0, col0;
  tile_origin(w - p * num_wg, nbr, gr, row0, col0);
  if (col0 >= n) return;
  const int k0 = p * kseg, kc = min(kseg, K_pad - k0);
  const int64_t off = (int64_t)k0 * n_pad, plane = (int64_t)n_pad * n_pad;
  hs_tile3m<4, true>(sm, W + off, WL + off, Y + off, kc, n_pad, n_pad, row0, col0, n, n, true, Hp + p * plane,
                     Sp + p * plane, n_pad);
}

__global__ void __launch_bounds__(256) k_sk_reduce(const d2* __restrict__ Hp, const d2* __restrict__ Sp, int ns,
                                                   int n, int n_pad, d2* __restrict__ H, d2* __restrict__ S,
                                                   int64_t ldh) {
  const int row = blockIdx.y;
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= n || col < row) return;
  const int64_t plane = (int64_t)n_pad * n_pad, e = (int64_t)row * n_pad + col;
  d2 h = Hp[e], sv = Sp[e];
  for (int p = 1; p < ns; ++p) {
    h += Hp[p * plane + e];
    sv += Sp[p * plane + e];
  }
  H[(int64_t)row * ldh + col] = h;
  S[(int64_t)row * ldh + col] = sv;
}

// Stream-K form of the 8-wave contraction: the units (tile t, 16-row chunk of the stacked
// index), tile-major, are dealt to nsh workgroups in equal contiguous shares, so every
// workgroup does the same number of MFMAs whatever the tile count.  A share holds the end of
// one tile, whole tiles and the start of another: whole tiles are stored into H and S, the
// piece a share starts with into its slot 0 and the piece it ends with into its slot 1
// (128 x 64 each, in Hp and Sp), and k_stream_fixup adds the pieces of each shared tile in
// chunk order, so results repeat bitwise.  Share c: units [units c / nsh, units (c + 1) / nsh).
__device__ inline int64_t stream_start(int64_t units, int nsh, int c) { return units * c / nsh; }
// the share holding unit u
__device__ inline int stream_share(int64_t units, int nsh, int64_t u) { return (int)(((u + 1) * nsh - 1) / units); }

__global__ void __launch_bounds__(512, 1) k_hs_fp64_stream(const d2* __restrict__ W, const d2* __restrict__ WL,
                                                           const d2* __restrict__ Y, int K_pad, int n, int n_pad,
                                                           int nbr, int num_tiles, int nsh, int gr,
                                                           d2* __restrict__ H, d2* __restrict__ S, int64_t ldh,
                                                           d2* __restrict__ Hp, d2* __restrict__ Sp) {
  __shared__ Smem sm;
  const int x = blockIdx.x % kXcds;
  int start, len;
  xcd_range(x, nsh, start, len);
  const int c = start + blockIdx.x / kXcds;  // consecutive shares, neighbouring tiles, on one XCD
  const int nk = K_pad / BK;
  const int64_t units = (int64_t)num_tiles * nk;
  const int64_t u0 = stream_start(units, nsh, c), u1 = stream_start(units, nsh, c + 1);
  for (int64_t u = u0; u < u1;) {
    const int t = (int)(u / nk);
    const int k0 = (int)(u - (int64_t)t * nk);
    const int k1 = (int)min((int64_t)nk, k0 + (u1 - u));
    // The tile routine's first copies go to LDS buffer 0, which the previous piece may still
    // be reading (its last chunk is there when its chunk count is odd).
    if (u != u0) __syncthreads();
    int row0, col0;
    tile_origin(t, nbr, gr, row0, col0);
    if (col0 < n) {  // uniform across the workgroup
      if (k0 == 0 && k1 == nk) {
        hs_tile3m<4, true>(sm, W, WL, Y, K_pad, n_pad, n_pad, row0, col0, n, n, true, H, S, ldh);
      } else {
        // element (row, col) of the piece at slot + (row - row0) * BN + (col - col0)
        const int64_t slot = (int64_t)(2 * c + (u == u0 ? 0 : 1)) * BM * BN - ((int64_t)row0 * BN + col0);
        const int64_t off = (int64_t)k0 * BK * n_pad;
        hs_tile3m<4, true>(sm, W + off, WL + off, Y + off, (k1 - k0) * BK, n_pad, n_pad, row0, col0, n, n, true,
                           (d2*)((uintptr_t)Hp + slot * (int64_t)sizeof(d2)),
                           (d2*)((uintptr_t)Sp + slot * (int64_t)sizeof(d2)), BN);
      }
    }
    u = (int64_t)t * nk + k1;
  }
}

// One workgroup per tile: a tile that lies in one share was stored whole; a shared one is the
// sum, in share (= chunk) order, of its pieces: slot 0 of the shares that start inside it,
// slot 1 of the one that starts before it.  Stored: row < n, col < n, col >= row.
__global__ void __launch_bounds__(256) k_stream_fixup(int K_pad, int n, int nbr, int num_tiles, int nsh, int gr,
                                                      const d2* __restrict__ Hp, const d2* __restrict__ Sp,
                                                      d2* __restrict__ H, d2* __restrict__ S, int64_t ldh) {
  const int t = blockIdx.x;
  const int nk = K_pad / BK;
  const int64_t units = (int64_t)num_tiles * nk;
  const int c0 = stream_share(units, nsh, (int64_t)t * nk), c1 = stream_share(units, nsh, (int64_t)t * nk + nk - 1);
  if (c0 == c1) return;
  int row0, col0;
  tile_origin(t, nbr, gr, row0, col0);
  if (col0 >= n) return;
  for (int e = threadIdx.x; e < BM * BN; e += 256) {
    const int row = row0 + e / BN, col = col0 + e % BN;
    if (row >= n || col >= n || col < row) continue;
    d2 h = d2{0.0, 0.0}, sv = d2{0.0, 0.0};
    for (int c = c0; c <= c1; ++c) {
      const int slot = 2 * c + (stream_start(units, nsh, c) >= (int64_t)t * nk ? 0 : 1);
      h += Hp[(int64_t)slot * BM * BN + e];
      sv += Sp[(int64_t)slot * BM * BN + e];
    }
    H[(int64_t)row * ldh + col] = h;
    S[(int64_t)row * ldh + col] = sv;
  }
}

template <int WR>
__global__ void __launch_bounds__(128 * WR, 1) k_hs_fp64_batch(const d2* __restrict__ ws, const double* __restrict__ lam,
                                                           int K_pad, const BatchMeta* __restrict__ meta, int n_k,
                                                           int total, int gr, d2* __restrict__ H,
                                                           d2* __restrict__ S) {
  __shared__ Smem sm;
  const int x = blockIdx.x % kXcds;
  const int per_xcd = gridDim.x / kXcds;  // the grid is a multiple of the XCD count
  int start, len;
  xcd_range(x, total, start, len);
  bool computed = false;  // a tile has been computed by this workgroup
  for (int i = blockIdx.x / kXcds; i < len; i += per_xcd) {
    const int t = start + i;
    int lo = 0, hi = n_k - 1;  // last k with tile_start <= t
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (meta[mid].tile_start <= t) lo = mid;
      else hi = mid - 1;
    }
    const BatchMeta m = meta[lo];
    int row0, col0;
    tile_origin(t - m.tile_start, m.nbr, gr, row0, col0);
    if (col0 >= m.n) continue;  // uniform across the workgroup
    // The tile routine's first copies go to LDS buffer 0, which the previous tile may still be
    // reading (its last chunk is there when the chunk count K_pad / 16 is odd).
    if (computed) __syncthreads();
    computed = true;
    if constexpr (WR == 4)
      hs_tile3m<WR, true>(sm, ws + m.w_off, ws + m.wl_off, ws + m.y_off, K_pad, m.n_pad, m.n_pad, row0, col0, m.n,
                          m.n, true, H + m.out_off, S + m.out_off, m.n);
    else
      hs_tile<WR, false>(sm, ws + m.w_off, ws + m.y_off, lam, K_pad, m.n, m.n_pad, row0, col0, H + m.out_off,
                         S + m.out_off, m.n);
  }
}

// Adjoint products P_H = W gH and P_S = W gS ([K_pad][n_pad]) with the same tile
// routine: tile rows k (128), columns G (64), contraction over G'.  The left operand
// is W^T (rows G', k contiguous, Kt = K_pad rounded to 128, zeros past K_pad), the
// right ones gS and gH zero-padded to n_pad x n_pad, so every copy is in bounds and
// the pads add nothing.  Full tiles, row-major tile order dealt to the XCDs in
// contiguous ranges (the tiles an XCD runs together share their W^T strip).
__global__ void __launch_bounds__(512, 1) k_pgemm3m(const d2* __restrict__ WT, const d2* __restrict__ gSp,
                                                  const d2* __restrict__ gHp, int Kt, int K_pad, int n_pad, int ncb,
                                                  int num_wg, d2* __restrict__ PH, d2* __restrict__ PS) {
  __shared__ Smem sm;
  const int x = blockIdx.x % kXcds;
  int start, len;
  xcd_range(x, num_wg, start, len);
  const int w = start + blockIdx.x / kXcds;
  const int rb = w / ncb, cb = w % ncb;
  hs_tile3m<4, false>(sm, WT, gSp, gHp, n_pad, Kt, n_pad, rb * BM, cb * BN, K_pad, n_pad, false, PH, PS, n_pad);
}

// Per-atom T products Y_a = T_t W_a on the same tile routine (plain products): tile
// rows r of Y_a (128), the routine's two outputs are two adjacent 64-column halves of
// a 128-column block (both share the staged T), contraction over the atom's rows k in
// 16-row chunks.  TT: per type T^T zero-padded to [Kc][MP] (Kc = round16(2N_L),
// MP = round128(2N_L)); rows of a chunk past 2N_L read the next atom's rows of W (or
// the zero rows past K, at least 15 of them) against zero rows of TT.
__global__ void __launch_bounds__(512, 1) k_tprod3m(CellArgs c, const d2* __restrict__ TT, const d2* __restrict__ W,
                                                  d2* __restrict__ Y, int n_pad, int Kc, int MP) {
  __shared__ Smem sm;
  const int atom = blockIdx.z;
  int t = 0;
  while (t + 1 < c.n_types && atom >= c.type_start[t + 1]) ++t;
  const int M = 2 * c.n_l;
  const d2* Wa = W + (int64_t)atom * M * n_pad;
  d2* Ya = Y + (int64_t)atom * M * n_pad;
  const int row0 = blockIdx.y * BM, col0 = blockIdx.x * 2 * BN;
  hs_tile3m<4, false>(sm, TT + (int64_t)t * Kc * MP, Wa, Wa + BN, Kc, MP, n_pad, row0, col0, M, n_pad, false, Ya + BN,
                      Ya, n_pad);
}

// Real-symmetric contraction on whole 128 x 128 super-tiles: Re(W^H Y) and
// Re(W^H lam W) keep two of the four real MFMAs per complex multiply-add, so
// with the 128 x 64 tile above a wave would read twice the LDS per MFMA.
// Here the tile is 128 x 128 and 8 rows are staged per chunk, copied straight
// into double-buffered LDS: 8 waves of 32 x 64 (2 x 4 MFMA blocks), the same
// MFMA work and LDS reads per chunk as the complex kernel.
constexpr int RN = 128, RK = 8;

struct RSmem {
  d2 L[2][RK][BM];
  d2 R[2][RK][RN];
  d2 Y[2][RK][RN];
};

__global__ void __launch_bounds__(512, 1) k_hs_real(const d2* __restrict__ W, const d2* __restrict__ WL,
                                                    const d2* __restrict__ Y, int K_pad, int n, int n_pad, int nbr,
                                                    int num_wg, int gr, double* __restrict__ H,
                                                    double* __restrict__ S, int64_t ldh) {
  __shared__ RSmem sm;
  const int x = blockIdx.x % kXcds;
  int start, len;
  xcd_range(x, num_wg, start, len);
  const int w = start + blockIdx.x / kXcds;
  int bi, bj;
  if (gr > 0) grouped_decode(w, nbr, gr, bi, bj);
  else tri_decode(w, nbr, bi, bj);
  const int row0 = bi * BM, col0 = bj * RN;
  if (col0 >= n) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;  // rows wr*32, columns wc*64

  // Staging straight into LDS: 48 copies of 1 KB (64 elements) per 8-row chunk, wave w
  // takes j = w + 8 i: copies 0..15 are W at the tile rows, 16..31 lam W (prepared in
  // HBM) and 32..47 Y at the tile columns; copy j covers row (j % 16) / 2, half j % 2.
  const d2* src0[6];
  int dst[6];  // d2 offset in buffer 0 of sm (L, R, Y are consecutive members)
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int j = wave + 8 * i, r = (j & 15) >> 1, half = j & 1;
    if (i < 2) {
      src0[i] = W + (int64_t)r * n_pad + row0 + half * 64;
      dst[i] = r * BM + half * 64;
    } else if (i < 4) {
      src0[i] = WL + (int64_t)r * n_pad + col0 + half * 64;
      dst[i] = 2 * RK * BM + r * RN + half * 64;
    } else {
      src0[i] = Y + (int64_t)r * n_pad + col0 + half * 64;
      dst[i] = 2 * RK * BM + 2 * RK * RN + r * RN + half * 64;
    }
  }
  d2* base = &sm.L[0][0][0];
  auto issue = [&](int c, int buf) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const int off = dst[i] + buf * (i < 2 ? RK * BM : RK * RN);
      __builtin_amdgcn_global_load_lds((const void*)(src0[i] + (int64_t)c * RK * n_pad + lane),
                                       (lds_ptr)(base + off), 16, 0, 0);
    }
  };

  d4 hr[2][4], sr[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) hr[i][j] = sr[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int nchunks = K_pad / RK;
  issue(0, 0);
  for (int c = 0; c < nchunks; ++c) {
    const int b = c & 1;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of chunk c have landed
    __syncthreads();                // everyone's have, and buffer b^1 is free
    if (c + 1 < nchunks) issue(c + 1, b ^ 1);
#pragma unroll
    for (int ks = 0; ks < RK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double ar[2], ai[2], yre[4], yim[4], wre[4], wim[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const d2 a = sm.L[b][kk][wr * 32 + i * 16 + (lane & 15)];
        ar[i] = a.x; ai[i] = a.y;
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const d2 yv = sm.Y[b][kk][wc * 64 + j * 16 + (lane & 15)];
        const d2 wv = sm.R[b][kk][wc * 64 + j * 16 + (lane & 15)];
        yre[j] = yv.x; yim[j] = yv.y; wre[j] = wv.x; wim[j] = wv.y;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) hr[i][j] = MFMA(ar[i], yre[j], hr[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) sr[i][j] = MFMA(ar[i], wre[j], sr[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) hr[i][j] = MFMA(ai[i], yim[j], hr[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) sr[i][j] = MFMA(ai[i], wim[j], sr[i][j]);
    }
  }

  // D layout of the 16x16 f64 MFMA: lane l, element q -> row l/16 + 4q, column l%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + wr * 32 + i * 16 + (lane >> 4) + 4 * q;
        const int col = col0 + wc * 64 + j * 16 + (lane & 15);
        if (row < n && col < n && col >= row) {
          const int64_t o = (int64_t)row * ldh + col;
          H[o] = hr[i][j][q];
          S[o] = sr[i][j][q];
        }
      }
}

}  // namespace

int hs_tiles(int n_pad) {
  const int nbr = n_pad / BM;
  return nbr * (nbr + 1);
}

hipError_t launch_tprod3m(const CellArgs& c, const double2* TT, const double2* W, double2* Y, int n_pad,
                          hipStream_t s) {
  const int M = 2 * c.n_l;
  if (n_pad % (2 * BN)) return hipErrorInvalidValue;
  dim3 grid(n_pad / (2 * BN), tprod_mp(M) / BM, c.n_atoms);
  hipLaunchKernelGGL(k_tprod3m, grid, dim3(512), 0, s, c, (const d2*)TT, (const d2*)W, (d2*)Y, n_pad, tprod_kc(M),
                     tprod_mp(M));
  return hipGetLastError();
}

hipError_t launch_pgemm3m(const double2* WT, const double2* gSp, const double2* gHp, int Kt, int K_pad, int n_pad,
                          double2* PH, double2* PS, hipStream_t s) {
  if (Kt % BM || n_pad % BN) return hipErrorInvalidValue;
  const int ncb = n_pad / BN, num_wg = ncb * (Kt / BM);
  hipLaunchKernelGGL(k_pgemm3m, dim3(num_wg), dim3(512), 0, s, (const d2*)WT, (const d2*)gSp, (const d2*)gHp, Kt,
                     K_pad, n_pad, ncb, num_wg, (d2*)PH, (d2*)PS);
  return hipGetLastError();
}

hipError_t launch_hs_fp64(const double2* W, const double2* WL, const double2* Y, const double* lam, int K_pad, int n,
                          int n_pad, int gr, int waves, double2* H, double2* S, int64_t ldh, hipStream_t s) {
  const int nbr = n_pad / BM;
  const int num_wg = hs_tiles(n_pad);  // two 128 x 64 tiles per upper-triangle 128 x 128 super-tile
  if (waves == 8)
    hipLaunchKernelGGL((k_hs_fp64<4, false>), dim3(num_wg), dim3(512), 0, s, (const d2*)W, (const d2*)WL,
                       (const d2*)Y, lam, K_pad, n, n_pad, nbr, num_wg, gr, (void*)H, (void*)S, ldh);
  else
    hipLaunchKernelGGL((k_hs_fp64<2, false>), dim3(num_wg), dim3(256), 0, s, (const d2*)W, (const d2*)WL,
                       (const d2*)Y, lam, K_pad, n, n_pad, nbr, num_wg, gr, (void*)H, (void*)S, ldh);
  return hipGetLastError();
}

int hs_stream_shares(int n_pad, int K_pad, int num_cus) {
  // time model, in stacked rows: a workgroup costs its rows plus about 128 per tile piece (the
  // pipeline start and the stores).  One pass: rounds of whole tiles on the compute units;
  // stream-K: the largest share, whose units span whole tiles and up to two partial ones.
  const int tiles = hs_tiles(n_pad);
  if (tiles >= 4 * num_cus || num_cus < 1) return 0;
  const int nk = K_pad / BK;
  const int64_t units = (int64_t)tiles * nk;
  const int nsh = (int)std::min<int64_t>(num_cus, units / 16);  // shares of at least 16 chunks (256 rows)
  if (nsh < 2) return 0;
  const double one_pass = std::ceil((double)tiles / num_cus) * (K_pad + 128.0);
  const double share = std::ceil((double)units / nsh);
  const double stream = share * BK + 128.0 * (std::ceil(share / nk) + 1.0);
  return stream < one_pass ? nsh : 0;
}

size_t hs_stream_slot_elems(int nsh) { return (size_t)2 * nsh * BM * BN; }

// The stream-K units follow one fixed tile order (super-rows 8 at a time): where the shares cut
// tiles, and so the rounding, must not depend on the tile-order option.
constexpr int kStreamGroup = 8;

int hs_split_rows(int K_pad, int ns) { return (int)round_up((K_pad + ns - 1) / ns, BK); }

hipError_t launch_hs_fp64_sk(const double2* W, const double2* WL, const double2* Y, int K_pad, int ns, int n,
                             int n_pad, int gr, double2* Hp, double2* Sp, hipStream_t s) {
  const int nbr = n_pad / BM;
  const int num_wg = hs_tiles(n_pad), total = num_wg * ns;
  const int kseg = hs_split_rows(K_pad, ns);
  if (K_pad % BK || kseg * (ns - 1) >= K_pad) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_hs_fp64_sk, dim3(total), dim3(512), 0, s, (const d2*)W, (const d2*)WL, (const d2*)Y, K_pad,
                     kseg, n, n_pad, nbr, num_wg, total, gr, (d2*)Hp, (d2*)Sp);
  return hipGetLastError();
}

hipError_t launch_hs_fp64_stream(const double2* W, const double2* WL, const double2* Y, int K_pad, int nsh, int n,
                                 int n_pad, double2* H, double2* S, int64_t ldh, double2* Hp, double2* Sp,
                                 hipStream_t s) {
  const int gr = kStreamGroup;
  const int nbr = n_pad / BM;
  const int num_tiles = hs_tiles(n_pad);
  if (K_pad % BK || nsh < 1 || (int64_t)num_tiles * (K_pad / BK) < nsh) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_hs_fp64_stream, dim3(nsh), dim3(512), 0, s, (const d2*)W, (const d2*)WL, (const d2*)Y, K_pad,
                     n, n_pad, nbr, num_tiles, nsh, gr, (d2*)H, (d2*)S, ldh, (d2*)Hp, (d2*)Sp);
  return hipGetLastError();
}

hipError_t launch_stream_fixup(int K_pad, int nsh, int n, int n_pad, const double2* Hp, const double2* Sp,
                               double2* H, double2* S, int64_t ldh, hipStream_t s) {
  const int gr = kStreamGroup;
  const int nbr = n_pad / BM;
  const int num_tiles = hs_tiles(n_pad);
  hipLaunchKernelGGL(k_stream_fixup, dim3(num_tiles), dim3(256), 0, s, K_pad, n, nbr, num_tiles, nsh, gr,
                     (const d2*)Hp, (const d2*)Sp, (d2*)H, (d2*)S, ldh);
  return hipGetLastError();
}

hipError_t launch_sk_reduce(const double2* Hp, const double2* Sp, int ns, int n, int n_pad, double2* H, double2* S,
                            int64_t ldh, hipStream_t s) {
  hipLaunchKernelGGL(k_sk_reduce, dim3((n + 255) / 256, n), dim3(256), 0, s, (const d2*)Hp, (const d2*)Sp, ns, n,
                     n_pad, (d2*)H, (d2*)S, ldh);
  return hipGetLastError();
}

hipError_t launch_hs_fp64_real(const double2* W, const double2* WL, const double2* Y, const double* lam, int K_pad,
                               int n, int n_pad, int gr, int waves, double* H, double* S, int64_t ldh, hipStream_t s) {
  const int nbr = n_pad / BM;
  const int num_wg = hs_tiles(n_pad);
  if (K_pad % RK) return hipErrorInvalidValue;
  if (waves == 8)  // whole 128 x 128 super-tiles
    hipLaunchKernelGGL(k_hs_real, dim3(num_wg / 2), dim3(512), 0, s, (const d2*)W, (const d2*)WL, (const d2*)Y, K_pad,
                       n, n_pad, nbr, num_wg / 2, gr, H, S, ldh);
  else
    hipLaunchKernelGGL((k_hs_fp64<2, true>), dim3(num_wg), dim3(256), 0, s, (const d2*)W, (const d2*)WL,
                       (const d2*)Y, lam, K_pad, n, n_pad, nbr, num_wg, gr, (void*)H, (void*)S, ldh);
  return hipGetLastError();
}

hipError_t launch_hs_fp64_batch(const double2* ws, const double* lam, int K_pad, const BatchMeta* meta, int n_k,
                                int total, int grid, int gr, int waves, double2* H, double2* S, hipStream_t s) {
  if (waves == 8)
    hipLaunchKernelGGL(k_hs_fp64_batch<4>, dim3(grid), dim3(512), 0, s, (const d2*)ws, lam, K_pad, meta, n_k, total,
                       gr, (d2*)H, (d2*)S);
  else
    hipLaunchKernelGGL(k_hs_fp64_batch<2>, dim3(grid), dim3(256), 0, s, (const d2*)ws, lam, K_pad, meta, n_k, total,
                       gr, (d2*)H, (d2*)S);
  return hipGetLastError();
}

}  // namespace hsb
