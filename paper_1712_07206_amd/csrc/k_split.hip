// Split-precision (Ozaki-style) form of the H/S contraction.
//
// Every operand column (one G: the vector over the stacked index k) is scaled
// by a power of two 2^e_G with max_k |Re|, |Im| < 2^e_G, then cut into S
// integer slices of 8 bits each:
//     x / 2^e = sum_{s=0}^{S-1} q_s 2^{-8(s+1)} + r,   |q_0| <= 256, |q_s| <= 128, |r| <= 2^{-8S-1}
// (round-to-nearest at each step, every step exact in FP64).  The slices are
// integers of at most 8 significant bits, hence exact in BF16 and FP16.  The
// product conj(L)^T R is then
//     2^{e_L(G') + e_R(G)} sum_d 2^{-8(d+2)} sum_{s+t=d} conj(L_s)^T R_t,   d < S,
// the pairs with s + t >= S being dropped (they are below the truncation).
// Slice products run on v_mfma_f32_16x16x32_{bf16,f16}; each level d has its
// own FP32 accumulator, which stays an exact integer while it sums at most 64
// stacked rows (|Re| <= 64 * 2 * 2^16.8 < 2^24); it is converted and added into
// the FP64 accumulator every 32 rows.  The level sums and the final scaling are
// FP64.
//
// Slice layout (16-byte units of 8 consecutive k): unit ((p * NB + b) * QK + q) * 64 + g
// holds plane p (= 2 s + {0: Re, 1: Im}), G = 64 b + g, k = 8 q .. 8 q + 7, so one
// 32-row chunk of a 64-column block is 4 KB contiguous.
#include "hs_internal.h"
#include "tiles.h"

namespace hsb {

namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// ---- column scales -------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_colmax(const d2* __restrict__ W, const d2* __restrict__ Y,
                                                const double* __restrict__ lam, int K, int n_pad,
                                                unsigned long long* __restrict__ mx) {
  const int G = blockIdx.x * 256 + threadIdx.x;
  if (G >= n_pad) return;
  const int k0 = blockIdx.y * 512;
  const int k1 = min(k0 + 512, K);
  double mw = 0.0, ms = 0.0, my = 0.0;
  for (int k = k0; k < k1; ++k) {
    const d2 w = W[(int64_t)k * n_pad + G];
    const d2 y = Y[(int64_t)k * n_pad + G];
    const double aw = fmax(fabs(w.x), fabs(w.y));
    mw = fmax(mw, aw);
    ms = fmax(ms, lam[k] * aw);
    my = fmax(my, fmax(fabs(y.x), fabs(y.y)));
  }
  // non-negative doubles order like their bit patterns
  atomicMax(&mx[G], (unsigned long long)__double_as_longlong(mw));
  atomicMax(&mx[n_pad + G], (unsigned long long)__double_as_longlong(ms));
  atomicMax(&mx[2 * n_pad + G], (unsigned long long)__double_as_longlong(my));
}

__global__ void __launch_bounds__(256) k_zero_u64(unsigned long long* __restrict__ a, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) a[i] = 0ull;
}

// scale[i] = 2^e with max < 2^e (frexp), 1 for an all-zero column
__global__ void __launch_bounds__(256) k_colscale(const unsigned long long* __restrict__ mx, int count,
                                                  double* __restrict__ scale) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const double m = __longlong_as_double((long long)mx[i]);
  int e = 0;
  if (m > 0.0) (void)frexp(m, &e);
  scale[i] = ldexp(1.0, e);
}

// ---- slicing ---------------------------------------------------------------------------
template <typename T>
__device__ inline unsigned short to_bits(double q);
template <>
__device__ inline unsigned short to_bits<__bf16>(double q) {
  const __bf16 v = (__bf16)(float)q;  // q: an integer |q| <= 256 times a power of two: exact
  return __builtin_bit_cast(unsigned short, v);
}
template <>
__device__ inline unsigned short to_bits<_Float16>(double q) {
  const _Float16 v = (_Float16)(float)q;
  return __builtin_bit_cast(unsigned short, v);
}

// One thread per (column G, 8-row group q); op 0: W, 1: lam W, 2: Y.
template <typename T, int S>
__global__ void __launch_bounds__(256) k_slice(const d2* __restrict__ X, const double* __restrict__ lam, int use_lam,
                                               int K, int n_pad, int QK, const double* __restrict__ scale,
                                               int prescale, u4* __restrict__ out) {
  const int g = threadIdx.x & 63;
  const int q = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int b = blockIdx.x;
  const int G = b * 64 + g;
  if (q >= QK) return;
  const double inv = 1.0 / scale[G];  // a power of two: exact
  double re[8], im[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = q * 8 + j;
    d2 v = d2{0.0, 0.0};
    if (k < K) {
      v = X[(int64_t)k * n_pad + G];
      if (use_lam) v *= lam[k];
    }
    re[j] = v.x * inv;
    im[j] = v.y * inv;
  }
  const int NB = n_pad / 64;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    unsigned short hr[8], hi[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double tr = re[j] * 256.0, ti = im[j] * 256.0;
      const double qr = rint(tr), qi = rint(ti);
      re[j] = tr - qr;
      im[j] = ti - qi;
      // pre-scaled slices carry their level weight 2^{-8s} (exact: a power of two)
      const double w = prescale ? __builtin_ldexp(1.0, -8 * s) : 1.0;
      hr[j] = to_bits<T>(qr * w);
      hi[j] = to_bits<T>(qi * w);
    }
    u4 ur, ui;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      ur[w] = (unsigned)hr[2 * w] | ((unsigned)hr[2 * w + 1] << 16);
      ui[w] = (unsigned)hi[2 * w] | ((unsigned)hi[2 * w + 1] << 16);
    }
    out[((int64_t)((2 * s) * NB + b) * QK + q) * 64 + g] = ur;
    out[((int64_t)((2 * s + 1) * NB + b) * QK + q) * 64 + g] = ui;
  }
}

// ---- slice contraction -----------------------------------------------------------------
constexpr int SBM = 128, SBN = 64, SNT = 256;
template <typename T>
__device__ inline f4 slice_mfma(u4 a, u4 b, f4 c);
template <>
__device__ inline f4 slice_mfma<__bf16>(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}
template <>
__device__ inline f4 slice_mfma<_Float16>(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
}

// Output tile 128 (G') x 64 (G); 4 waves, each 64 x 32 (4 x 2 MFMA blocks).  Per
// 32-row chunk the slices of both operand tiles sit in LDS (single buffer, the
// next chunk prefetched into registers); the levels are taken one at a time,
// each with its FP32 accumulators, which are added into the FP64 ones at the
// end of the level (32 rows: exact).
template <typename T, int S>
__global__ void __launch_bounds__(SNT, 1) k_hs_split(const u4* __restrict__ Ls, const u4* __restrict__ Rs,
                                                     const double* __restrict__ scL, const double* __restrict__ scR,
                                                     int QK, int n, int n_pad, int nbr, int num_wg,
                                                     d2* __restrict__ C) {
  constexpr int P = 2 * S;                   // planes per operand
  constexpr int LU = P * 2 * 4 * 64;         // left units per 32-row chunk
  constexpr int RU = P * 4 * 64;             // right units per chunk
  constexpr int PER = (LU + RU) / SNT;       // units staged per thread
  static_assert((LU + RU) % SNT == 0, "staging map");
  __shared__ u4 lds[LU + RU];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;   // rows wr*64, columns wc*32
  const int x = blockIdx.x % kXcds;
  int start, len;
  xcd_range(x, num_wg, start, len);
  const int w = start + blockIdx.x / kXcds;
  int bi, sj;
  tri_decode(w >> 1, nbr, bi, sj);
  const int row0 = bi * SBM, col0 = sj * SBM + (w & 1) * SBN;
  if (col0 >= n) return;
  const int NB = n_pad / 64;
  const int bL = row0 / 64, bR = col0 / 64;

  d2 a64[4][2][4];  // [i][j][element] (re, im)
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) a64[i][j][e] = d2{0.0, 0.0};

  u4 pf[PER];
  const int nchunks = QK / 4;
#define SP_GLOAD(q0)                                                                    \
  do {                                                                                  \
    _Pragma("unroll") for (int r = 0; r < PER; ++r) {                                   \
      const int u = tid + SNT * r;                                                      \
      if (u < LU) {                                                                     \
        const int p = u >> 9, rem = u & 511;                                            \
        pf[r] = Ls[((int64_t)(p * NB + bL + (rem >> 8)) * QK + (q0) + ((rem >> 6) & 3)) * 64 + (rem & 63)]; \
      } else {                                                                          \
        const int v = u - LU;                                                           \
        const int p = v >> 8;                                                           \
        pf[r] = Rs[((int64_t)(p * NB + bR) * QK + (q0) + ((v >> 6) & 3)) * 64 + (v & 63)]; \
      }                                                                                 \
    }                                                                                   \
  } while (0)

  SP_GLOAD(0);
  const int qq = lane >> 4;
  for (int c = 0; c < nchunks; ++c) {
    __syncthreads();  // the previous chunk's reads are done
#pragma unroll
    for (int r = 0; r < PER; ++r) lds[tid + SNT * r] = pf[r];
    __syncthreads();
    if (c + 1 < nchunks) SP_GLOAD((c + 1) * 4);
#pragma unroll 1
    for (int d = 0; d < S; ++d) {
      f4 are[4][2], aim[4][2];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          are[i][j] = f4{0.f, 0.f, 0.f, 0.f};
          aim[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll 1
      for (int s = 0; s <= d; ++s) {
        const int t = d - s;
        u4 lr[4], li[4], rr[2], ri[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // row g' = wr*64 + i*16 + lane%16 of the tile: 64-block wr, column within it
          const int gg = i * 16 + (lane & 15);
          lr[i] = lds[(((2 * s) * 2 + wr) * 4 + qq) * 64 + gg];
          li[i] = lds[(((2 * s + 1) * 2 + wr) * 4 + qq) * 64 + gg];
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int g = wc * 32 + j * 16 + (lane & 15);
          rr[j] = lds[LU + ((2 * t) * 4 + qq) * 64 + g];
          ri[j] = lds[LU + ((2 * t + 1) * 4 + qq) * 64 + g];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) are[i][j] = slice_mfma<T>(lr[i], rr[j], are[i][j]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) aim[i][j] = slice_mfma<T>(lr[i], ri[j], aim[i][j]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) are[i][j] = slice_mfma<T>(li[i], ri[j], are[i][j]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const u4 ln = li[i] ^ u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
#pragma unroll
          for (int j = 0; j < 2; ++j) aim[i][j] = slice_mfma<T>(ln, rr[j], aim[i][j]);
        }
      }
      const double sc = __builtin_ldexp(1.0, -8 * (d + 2));
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            a64[i][j][e].x += sc * (double)are[i][j][e];
            a64[i][j][e].y += sc * (double)aim[i][j][e];
          }
    }
  }
#undef SP_GLOAD
  // D layout of the 16x16 f32 MFMA: lane l, element e -> row 4 (l/16) + e, column l%16
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = row0 + wr * 64 + i * 16 + 4 * (lane >> 4) + e;
        const int col = col0 + wc * 32 + j * 16 + (lane & 15);
        if (row < n && col < n && col >= row) {
          const double sc = scL[row] * scR[col];
          C[(int64_t)row * n + col] = a64[i][j][e] * sc;
        }
      }
}

// ---- BF16 contraction with folded levels (pre-scaled slices) ------------------------------
// Slice s is stored as q_s 2^{-8s}, so the product of pair (s, t) already carries
// its weight 2^{-8(s+t)}.  Four FP32 accumulator sets: levels 0, 1 and 2 each in
// their own set, where every partial sum over 64 rows is an exact multiple of
// 2^{-8d} below 2^{24-8d} (|level-2 row term| <= 2 (2^15 + 2^14 + 2^15) 2^-16), and
// all levels >= 3 in one set whose FP32 rounding is below 2^-40 of the leading
// term.  The sets are added into FP64 every 64 rows.  MFMA 32x32x16 (lane l: row
// l%32, k 8(l/32)..+7; output lane l, element r: column l%32, row 8(r/4) + 4(l/32) +
// r%4).  16-row chunks of the slices are copied straight into double-buffered LDS
// with global_load_lds_dwordx4 (no staging registers).  8 waves of 32 x 32 (two per
// SIMD) cover the 128 x 64 tile.
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __attribute__((address_space(3))) void* lds_ptr;

// scheduling groups (DS read = 0x100, MFMA = 0x008): reads of step K + 1, then the 4 (K + 1) MFMAs of step K
template <int K, int S>
__device__ __forceinline__ void split2_schedule() {
  if constexpr (K < S) {
    if constexpr (K + 1 < S) __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 4 * (K + 1), 0);
    split2_schedule<K + 1, S>();
  }
}

template <int S>
__global__ void __launch_bounds__(512, 1) k_hs_split2(const u4* __restrict__ Ls, const u4* __restrict__ Rs,
                                                      const double* __restrict__ scL, const double* __restrict__ scR,
                                                      int QK, int n, int n_pad, int nbr, int num_wg, int gr,
                                                      d2* __restrict__ C) {
  constexpr int P = 2 * S;        // planes per operand
  constexpr int CU = 384 * P;     // units per chunk: left P*2*2*64, right P*2*64
  constexpr int NI = 6 * P;       // 64-unit copies per chunk
  __shared__ u4 lds[2][CU];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: copy addresses stay scalar
  const int wr = wave >> 1, wc = wave & 1;  // rows wr*32, columns wc*32 (8 waves: 4 x 2)
  const int x = blockIdx.x % kXcds;
  int start, len;
  xcd_range(x, num_wg, start, len);
  const int w = start + blockIdx.x / kXcds;
  int row0, col0;
  tile_origin(w, nbr, gr, row0, col0);
  if (col0 >= n) return;
  const int NB = n_pad / 64;
  const int bL = row0 / 64, bR = col0 / 64;
  const int nchunks = QK / 2;

  // The copies of a chunk (64 units = 1 KB each): left (p, b, q) for j < 4P, right (p, q)
  // after; wave w takes j = w, w + 8, ...  A copy's source advances by 128 units per chunk.
  constexpr int NPW = (NI + 7) / 8;
  const u4* src0[NPW];
  int dst[NPW];
#pragma unroll
  for (int i = 0; i < NPW; ++i) {
    const int j = wave + 8 * i;
    src0[i] = Ls;  // unused when j >= NI
    dst[i] = 0;
    if (j >= NI) continue;
    if (j < 4 * P) {
      const int p = j >> 2, b = (j >> 1) & 1, qq = j & 1;
      src0[i] = Ls + ((int64_t)(p * NB + bL + b) * QK + qq) * 64;
      dst[i] = ((p * 2 + b) * 2 + qq) * 64;
    } else {
      const int jj = j - 4 * P;
      const int p = jj >> 1, qq = jj & 1;
      src0[i] = Rs + ((int64_t)(p * NB + bR) * QK + qq) * 64;
      dst[i] = 256 * P + (p * 2 + qq) * 64;
    }
  }
  auto issue = [&](int c, int buf) {
#pragma unroll
    for (int i = 0; i < NPW; ++i)
      if (wave + 8 * i < NI)
        __builtin_amdgcn_global_load_lds((const void*)(src0[i] + (int64_t)c * 128 + lane),
                                         (lds_ptr)(&lds[buf][dst[i]]), 16, 0, 0);
  };
  // The two waves that share a SIMD (w and w + 4) flush at chunks two apart, so one
  // converts while the other keeps the MFMA unit busy; every window stays <= 64 rows.
  const int fph = (wave >> 2) ? 2 : 0;

  f16v acc[4][2];  // [set][re, im]
  double a64[2][16];
#pragma unroll
  for (int r = 0; r < 16; ++r) a64[0][r] = a64[1][r] = 0.0;
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[st][0][r] = acc[st][1][r] = 0.f;

  issue(0, 0);
  const int q = lane >> 5, g32 = lane & 31;
  // row block of this wave: rows wr*32 .. of the 128-row tile = 64-block (wr >> 1), offset (wr & 1) * 32
  const int lrow = ((wr >> 1) * 2 + q) * 64 + (wr & 1) * 32 + g32;  // + p * 256 selects the plane
  const int rcol = 256 * P + q * 64 + wc * 32 + g32;                 // + p * 128 selects the plane
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of chunk c have landed
    __syncthreads();                // everyone's have, and buffer buf^1 is free
    if (c + 1 < nchunks) issue(c + 1, buf ^ 1);
    const u4* B = lds[buf];
    // Step k takes left slice si = S-1-k and right slice k, and runs every pair (si, t <= k):
    // the reads are spread over the chunk instead of all waiting up front.
    u4 rre[S], rim[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const int si = S - 1 - k;
      const u4 lr = B[lrow + (2 * si) * 256];
      const u4 li = B[lrow + (2 * si + 1) * 256];
      rre[k] = B[rcol + (2 * k) * 128];
      rim[k] = B[rcol + (2 * k + 1) * 128];
      const u4 ln = li ^ u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
#pragma unroll
      for (int ti = 0; ti <= k; ++ti) {
        const int st = si + ti < 3 ? si + ti : 3;
        const bf8 brr = __builtin_bit_cast(bf8, rre[ti]);
        const bf8 bri = __builtin_bit_cast(bf8, rim[ti]);
        acc[st][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, lr), brr, acc[st][0], 0, 0, 0);
        acc[st][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, lr), bri, acc[st][1], 0, 0, 0);
        acc[st][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, li), bri, acc[st][0], 0, 0, 0);
        acc[st][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf8, ln), brr, acc[st][1], 0, 0, 0);
      }
    }
    // schedule: the four reads of step k + 1 are issued ahead of the MFMAs of step k
    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
    split2_schedule<0, S>();
    if (((c + fph) & 3) == 3 || c + 1 == nchunks) {  // <= 64 rows: the exact sets are still exact
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double sre = 0.0, sim = 0.0;
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          sre += (double)acc[st][0][r];
          sim += (double)acc[st][1][r];
          acc[st][0][r] = 0.f;
          acc[st][1][r] = 0.f;
        }
        a64[0][r] += 0x1p-16 * sre;
        a64[1][r] += 0x1p-16 * sim;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = row0 + wr * 32 + 8 * (r >> 2) + 4 * q + (r & 3);
    const int col = col0 + wc * 32 + g32;
    if (row < n && col < n && col >= row) {
      const double sc = scL[row] * scR[col];
      C[(int64_t)row * n + col] = d2{a64[0][r] * sc, a64[1][r] * sc};
    }
  }
}

// ---- int8 slices ------------------------------------------------------------------------
// Seven-bit slices in signed bytes:
//     x / 2^e = sum_{s=0}^{S-1} q_s 2^{-6-7s} + r,   q_0 = rint(64 x), q_s = rint(128 r_{s-1}),
// so |q_s| <= 64 and |r| <= 2^{-7S}, every step exact in FP64.  Unit ((p * NB + b) * QK + q)
// * 64 + g holds plane p (= 2 s + {0: Re, 1: Im}), G = 64 b + g, k = 16 q .. 16 q + 15, one
// byte each, so a 32-row chunk of a 64-column block is 2 KB contiguous per plane.
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));

template <int S>
__global__ void __launch_bounds__(256) k_slice8(const d2* __restrict__ X, const double* __restrict__ lam,
                                                int use_lam, int K, int n_pad, int QK,
                                                const double* __restrict__ scale, u4* __restrict__ out) {
  const int g = threadIdx.x & 63;
  const int q = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int b = blockIdx.x;
  const int G = b * 64 + g;
  if (q >= QK) return;
  const double inv = 64.0 / scale[G];  // a power of two: exact
  double re[16], im[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int k = q * 16 + j;
    d2 v = d2{0.0, 0.0};
    if (k < K) {
      v = X[(int64_t)k * n_pad + G];
      if (use_lam) v *= lam[k];
    }
    re[j] = v.x * inv;
    im[j] = v.y * inv;
  }
  const int NB = n_pad / 64;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    u4 ur = u4{0u, 0u, 0u, 0u}, ui = u4{0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double qr = rint(re[j]), qi = rint(im[j]);
      re[j] = (re[j] - qr) * 128.0;
      im[j] = (im[j] - qi) * 128.0;
      ur[j >> 2] |= ((unsigned)(int)qr & 0xffu) << (8 * (j & 3));
      ui[j >> 2] |= ((unsigned)(int)qi & 0xffu) << (8 * (j & 3));
    }
    out[((int64_t)((2 * s) * NB + b) * QK + q) * 64 + g] = ur;
    out[((int64_t)((2 * s + 1) * NB + b) * QK + q) * 64 + g] = ui;
  }
}

// Bytewise negation of four signed bytes per word (no borrow crosses a byte).
__device__ __forceinline__ u4 neg_bytes(u4 x) {
  u4 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = (0x80808080u - (x[i] & 0x7f7f7f7fu)) ^ (~x[i] & 0x80808080u);
  return r;
}

__device__ __forceinline__ i16v mfma_i8(u4 a, u4 b, i16v c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(i4v, a), __builtin_bit_cast(i4v, b), c, 0, 0, 0);
}

// int8 contraction.  Tile, waves and staging as in k_hs_split2 (128 x 64 tile, 8 waves of
// 32 x 32, direct-to-LDS copies into double-buffered LDS), with 32-row chunks: a 16-byte
// unit holds 16 rows of one slice plane.  Pair (s, t) runs on v_mfma_i32_32x32x32_i8 into
// the int32 sum of its level d = s + t, which is exact: per row a channel adds two
// products of at most 64 * 64, and a level takes at most S pairs, so 32768 rows stay
// below 2^{13+15} S < 2^31 for S <= 6.  Every 32768 rows (and at the end) the levels are
// combined in FP64 with weights 2^{-12-7d} and the column scales, and added into C, which
// the same lane wrote at the previous flush.
constexpr int kFlush8 = 1024;  // chunks of 32 rows between flushes

// LDS reads that pair j (loop order: left slice si, then right slice ti < S - si) issues.
// Right slices 0 and 1 are read once per chunk, by the pairs (0, 0) and (0, 1), and kept;
// every other right slice is read by its pair; each left slice is read by its first pair.
template <int S>
constexpr int split8_reads(int j) {
  int idx = 0;
  for (int si = 0; si < S; ++si)
    for (int ti = 0; ti < S - si; ++ti, ++idx)
      if (idx == j) return (ti == 0 ? 2 : 0) + (ti >= 2 || si == 0 ? 2 : 0);
  return 0;
}

// scheduling groups (DS read = 0x100, MFMA = 0x008): the reads of pair j + 1, then the
// four MFMAs of pair j, so that two pairs' operands are live at a time
template <int S, int J, int M>
__device__ __forceinline__ void split8_schedule() {
  constexpr int NP = S * (S + 1) / 2;
  if constexpr (J < NP) {
    if constexpr (J + 1 < NP) __builtin_amdgcn_sched_group_barrier(0x100, split8_reads<S>(J + 1), 0);
    __builtin_amdgcn_sched_group_barrier(0x008, M, 0);
    split8_schedule<S, J + 1, M>();
  }
}

// REAL: C = Re(conj(L)^T R), one int32 channel per level (two MFMAs per pair: Re L Re R
// and Im L Im R), written to a real [n][n] array.
template <int S, bool REAL>
__global__ void __launch_bounds__(512, 1) k_hs_split8(const u4* __restrict__ Ls, const u4* __restrict__ Rs,
                                                      const double* __restrict__ scL, const double* __restrict__ scR,
                                                      int QK, int n, int n_pad, int nbr, int num_wg, int gr,
                                                      void* __restrict__ Cv) {
  constexpr int NCH = REAL ? 1 : 2;  // int32 channels per level
  constexpr int P = 2 * S;        // planes per operand
  constexpr int CU = 384 * P;     // units per chunk: left P*2*2*64, right P*2*64
  constexpr int NI = 6 * P;       // 64-unit copies per chunk
  __shared__ u4 lds[2][CU];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int x = blockIdx.x % kXcds;
  int start, len;
  xcd_range(x, num_wg, start, len);
  const int w = start + blockIdx.x / kXcds;
  int row0, col0;
  tile_origin(w, nbr, gr, row0, col0);
  if (col0 >= n) return;
  const int NB = n_pad / 64;
  const int bL = row0 / 64, bR = col0 / 64;
  const int nchunks = QK / 2;

  constexpr int NPW = (NI + 7) / 8;
  const u4* src0[NPW];
  int dst[NPW];
#pragma unroll
  for (int i = 0; i < NPW; ++i) {
    const int j = wave + 8 * i;
    src0[i] = Ls;
    dst[i] = 0;
    if (j >= NI) continue;
    if (j < 4 * P) {
      const int p = j >> 2, b = (j >> 1) & 1, qq = j & 1;
      src0[i] = Ls + ((int64_t)(p * NB + bL + b) * QK + qq) * 64;
      dst[i] = ((p * 2 + b) * 2 + qq) * 64;
    } else {
      const int jj = j - 4 * P;
      const int p = jj >> 1, qq = jj & 1;
      src0[i] = Rs + ((int64_t)(p * NB + bR) * QK + qq) * 64;
      dst[i] = 256 * P + (p * 2 + qq) * 64;
    }
  }
  auto issue = [&](int c, int buf) {
#pragma unroll
    for (int i = 0; i < NPW; ++i)
      if (wave + 8 * i < NI)
        __builtin_amdgcn_global_load_lds((const void*)(src0[i] + (int64_t)c * 128 + lane),
                                         (lds_ptr)(&lds[buf][dst[i]]), 16, 0, 0);
  };

  i16v acc[S][NCH];
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[d][ch][r] = 0;

  const int q = lane >> 5, g32 = lane & 31;
  const int lrow = ((wr >> 1) * 2 + q) * 64 + (wr & 1) * 32 + g32;
  const int rcol = 256 * P + q * 64 + wc * 32 + g32;
  // output element r of this lane: D layout of the 32 x 32 MFMA
  auto flush = [&](bool first) {
    // the tile origin is loop-invariant: an opaque copy keeps the output addresses and
    // scales from being hoisted out of the chunk loop (and held in registers through it)
    int rb = row0 + wr * 32 + 4 * q, cb = col0 + wc * 32 + g32;
    asm volatile("" : "+v"(rb), "+v"(cb));
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      double vre = 0.0, vim = 0.0;
#pragma unroll
      for (int d = 0; d < S; ++d) {
        vre += __builtin_ldexp((double)acc[d][0][r], -7 * d);
        acc[d][0][r] = 0;
        if constexpr (!REAL) {
          vim += __builtin_ldexp((double)acc[d][1][r], -7 * d);
          acc[d][1][r] = 0;
        }
      }
      const int row = rb + 8 * (r >> 2) + (r & 3);
      const int col = cb;
      if (row < n && col < n && col >= row) {
        const double sc = 0x1p-12 * scL[row] * scR[col];
        if constexpr (REAL) {
          double* C = (double*)Cv;
          double v = vre * sc;
          if (!first) v += C[(int64_t)row * n + col];
          C[(int64_t)row * n + col] = v;
        } else {
          d2* C = (d2*)Cv;
          d2 v = d2{vre * sc, vim * sc};
          if (!first) v += C[(int64_t)row * n + col];
          C[(int64_t)row * n + col] = v;
        }
      }
    }
  };

  if (nchunks == 0) {
    flush(true);
    return;
  }
  issue(0, 0);
  for (int c = 0; c < nchunks; ++c) {
    const int buf = c & 1;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (c + 1 < nchunks) issue(c + 1, buf ^ 1);
    const u4* B = lds[buf];
    // right slices 0 and 1 pair with all but one left slice: read once per chunk and kept
    const u4 rr0 = B[rcol], ri0 = B[rcol + 128];
    const u4 rr1 = B[rcol + 256], ri1 = B[rcol + 384];
#pragma unroll
    for (int si = 0; si < S; ++si) {
      const u4 lr = B[lrow + (2 * si) * 256];
      const u4 li = B[lrow + (2 * si + 1) * 256];
      u4 ln;
      if constexpr (!REAL) ln = neg_bytes(li);
      // the other right slices are re-read for every left slice (an opaque index keeps the
      // reads from being merged, which would hold all 2S right operands live through the chunk)
      int rc = rcol;
      asm volatile("" : "+v"(rc));
      const u4* BR = B + rc;
#pragma unroll
      for (int ti = 0; ti < S - si; ++ti) {
        const u4 rr = ti == 0 ? rr0 : ti == 1 ? rr1 : BR[(2 * ti) * 128];
        const u4 ri = ti == 0 ? ri0 : ti == 1 ? ri1 : BR[(2 * ti + 1) * 128];
        const int d = si + ti;
        if constexpr (REAL) {
          acc[d][0] = mfma_i8(lr, rr, acc[d][0]);
          acc[d][0] = mfma_i8(li, ri, acc[d][0]);
        } else {
          acc[d][0] = mfma_i8(lr, rr, acc[d][0]);
          acc[d][1] = mfma_i8(lr, ri, acc[d][1]);
          acc[d][0] = mfma_i8(li, ri, acc[d][0]);
          acc[d][1] = mfma_i8(ln, rr, acc[d][1]);
        }
      }
    }
    __builtin_amdgcn_sched_group_barrier(0x100, split8_reads<S>(0), 0);
    split8_schedule<S, 0, REAL ? 2 : 4>();
    if ((c + 1) % kFlush8 == 0 || c + 1 == nchunks) flush(c < kFlush8);
  }
}

template <bool REAL>
hipError_t launch_hs_split8(int S, const void* L, const void* R, const double* scL, const double* scR, int QK, int n,
                            int n_pad, int gr, void* C, hipStream_t s) {
  const int nbr = n_pad / SBM;
  const int num_wg = nbr * (nbr + 1);
  dim3 grid(num_wg), block(512);
  switch (S) {
    case 3: hipLaunchKernelGGL((k_hs_split8<3, REAL>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, gr, C); break;
    case 4: hipLaunchKernelGGL((k_hs_split8<4, REAL>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, gr, C); break;
    case 5: hipLaunchKernelGGL((k_hs_split8<5, REAL>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, gr, C); break;
    case 6: hipLaunchKernelGGL((k_hs_split8<6, REAL>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, gr, C); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_slices8(int S, const double2* X, const double* lam, int use_lam, int K, int n_pad, int QK,
                          const double* scale, void* out, hipStream_t s) {
  dim3 grid(n_pad / 64, (QK + 3) / 4);
  switch (S) {
    case 3: hipLaunchKernelGGL((k_slice8<3>), grid, dim3(256), 0, s, (const d2*)X, lam, use_lam, K, n_pad, QK, scale, (u4*)out); break;
    case 4: hipLaunchKernelGGL((k_slice8<4>), grid, dim3(256), 0, s, (const d2*)X, lam, use_lam, K, n_pad, QK, scale, (u4*)out); break;
    case 5: hipLaunchKernelGGL((k_slice8<5>), grid, dim3(256), 0, s, (const d2*)X, lam, use_lam, K, n_pad, QK, scale, (u4*)out); break;
    case 6: hipLaunchKernelGGL((k_slice8<6>), grid, dim3(256), 0, s, (const d2*)X, lam, use_lam, K, n_pad, QK, scale, (u4*)out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_hs_split2(int S, const void* L, const void* R, const double* scL, const double* scR, int QK, int n,
                            int n_pad, int gr, double2* C, hipStream_t s) {
  const int nbr = n_pad / SBM;
  const int num_wg = nbr * (nbr + 1);
  dim3 grid(num_wg), block(512);
  switch (S) {
    case 3: hipLaunchKernelGGL((k_hs_split2<3>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, gr, (d2*)C); break;
    case 4: hipLaunchKernelGGL((k_hs_split2<4>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, gr, (d2*)C); break;
    case 5: hipLaunchKernelGGL((k_hs_split2<5>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, gr, (d2*)C); break;
    case 6: hipLaunchKernelGGL((k_hs_split2<6>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, gr, (d2*)C); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_slices_t(int S, const double2* X, const double* lam, int use_lam, int K, int n_pad, int QK,
                           const double* scale, int prescale, void* out, hipStream_t s) {
  dim3 grid(n_pad / 64, (QK + 3) / 4);
  switch (S) {
    case 3: hipLaunchKernelGGL((k_slice<T, 3>), grid, dim3(256), 0, s, (const d2*)X, lam, use_lam, K, n_pad, QK, scale, prescale, (u4*)out); break;
    case 4: hipLaunchKernelGGL((k_slice<T, 4>), grid, dim3(256), 0, s, (const d2*)X, lam, use_lam, K, n_pad, QK, scale, prescale, (u4*)out); break;
    case 5: hipLaunchKernelGGL((k_slice<T, 5>), grid, dim3(256), 0, s, (const d2*)X, lam, use_lam, K, n_pad, QK, scale, prescale, (u4*)out); break;
    case 6: hipLaunchKernelGGL((k_slice<T, 6>), grid, dim3(256), 0, s, (const d2*)X, lam, use_lam, K, n_pad, QK, scale, prescale, (u4*)out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_hs_split_t(int S, const void* L, const void* R, const double* scL, const double* scR, int QK,
                             int n, int n_pad, double2* C, hipStream_t s) {
  const int nbr = n_pad / SBM;
  const int num_wg = nbr * (nbr + 1);
  dim3 grid(num_wg), block(SNT);
  switch (S) {
    case 3: hipLaunchKernelGGL((k_hs_split<T, 3>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, (d2*)C); break;
    case 4: hipLaunchKernelGGL((k_hs_split<T, 4>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, (d2*)C); break;
    case 5: hipLaunchKernelGGL((k_hs_split<T, 5>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, (d2*)C); break;
    case 6: hipLaunchKernelGGL((k_hs_split<T, 6>), grid, block, 0, s, (const u4*)L, (const u4*)R, scL, scR, QK, n, n_pad, nbr, num_wg, (d2*)C); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_split_scales(const double2* W, const double2* Y, const double* lam, int K, int n_pad,
                               unsigned long long* mx, double* scale, hipStream_t s) {
  const int count = 3 * n_pad;
  hipLaunchKernelGGL(k_zero_u64, dim3((count + 255) / 256), dim3(256), 0, s, mx, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colmax, dim3(n_pad / 256 + (n_pad % 256 ? 1 : 0), (K + 511) / 512), dim3(256), 0, s,
                     (const d2*)W, (const d2*)Y, lam, K, n_pad, mx);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colscale, dim3((count + 255) / 256), dim3(256), 0, s, (const unsigned long long*)mx, count,
                     scale);
  return hipGetLastError();
}

hipError_t launch_split_slices(int precision, int S, const double2* X, const double* lam, int use_lam, int K,
                               int n_pad, int QK, const double* scale, void* out, hipStream_t s) {
  if (precision == HSB_SPLIT_INT8) return launch_slices8(S, X, lam, use_lam, K, n_pad, QK, scale, out, s);
  // BF16 slices are stored pre-scaled for the level-folding contraction
  if (precision == HSB_SPLIT_BF16) return launch_slices_t<__bf16>(S, X, lam, use_lam, K, n_pad, QK, scale, 1, out, s);
  return launch_slices_t<_Float16>(S, X, lam, use_lam, K, n_pad, QK, scale, 0, out, s);
}

hipError_t launch_hs_split(int precision, int S, const void* L, const void* R, const double* scL, const double* scR,
                           int QK, int n, int n_pad, int gr, double2* C, hipStream_t s) {
  if (precision == HSB_SPLIT_INT8) return launch_hs_split8<false>(S, L, R, scL, scR, QK, n, n_pad, gr, C, s);
  if (precision == HSB_SPLIT_BF16) return launch_hs_split2(S, L, R, scL, scR, QK, n, n_pad, gr, C, s);
  return launch_hs_split_t<_Float16>(S, L, R, scL, scR, QK, n, n_pad, C, s);
}

hipError_t launch_hs_split8_real(int S, const void* L, const void* R, const double* scL, const double* scR, int QK,
                                 int n, int n_pad, int gr, double* C, hipStream_t s) {
  return launch_hs_split8<true>(S, L, R, scL, scR, QK, n, n_pad, gr, C, s);
}

}  // namespace hsb
