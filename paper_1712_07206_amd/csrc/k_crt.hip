// Split-precision contraction by residues (Chinese remainder theorem) on the int8 matrix
// cores, or on the BF16/FP16 matrix cores with the residues as 16-bit integers: the residue
// forms of the split path.
//
// Every operand column (one G: the vector over the stacked index k) is scaled by a
// power of two 2^f_G and rounded to Gaussian integers x' = rint(2^f x) (exact in
// FP64).  The integer product conj(L')^T R' of two such columns is represented by its
// residues modulo n pairwise coprime moduli m_i.  Each m_i is a power of a prime
// p = 1 (mod 4), so -1 has a square root j_i modulo m_i and the Gaussian integers
// modulo m_i split into two copies of Z/m_i:
//     z = x + i y  ->  (x + j y, x - j y)  (mod m),
// a ring isomorphism (its inverse: x = (u + v)/2, y = (u - v)/(2j)).  The conjugated
// product of two columns then costs two integer inner products per modulus instead of
// four:
//     P = sum_k (a_r - j a_i)_k (b_r + j b_i)_k,   Q = sum_k (a_r + j a_i)_k (b_r - j b_i)_k,
//     Re = (P + Q) / 2,   Im = (P - Q) / (2j)      (mod m),
// with the residues stored as signed bytes in [-(m-1)/2, (m-1)/2] and P, Q exact int32
// sums on v_mfma_i32_32x32x32_i8 (or as bfloat16/half integers with FP32 sums on
// v_mfma_f32_32x32x16_{bf16,f16}, exact below 2^24 and reduced modulo m every 1024 rows, so
// the residues, and H and S, are the same).  The column scaling keeps |Re|, |Im| of the integer
// product below M/2 (M = prod m_i) by Cauchy-Schwarz, so the residues fix it uniquely;
// it is recovered in FP64 as M * frac(sum_i r_i y_i / m_i), y_i = (M/m_i)^{-1} mod m_i,
// with y_i / m_i split into a part on a 2^-42 grid (whose weighted sum is exact) and a
// small remainder.  The only approximation is the rounding of the scaled operands to
// integers; at 11 moduli that keeps 40 bits of each column's 2-norm.
//
// Residue layout: 16-byte units of RU consecutive k (RU = 16 bytes, or 8 16-bit elements),
// chunk-major, a chunk being 4 units (64 rows of bytes, 32 of 16-bit elements):
// unit i * 2 NB QK * 64 + (((c * NB + b) * 2 + p) * 4 + qq) * 64 + g holds, for modulus i,
// plane p (0: x_r + j_i x_i, 1: x_r - j_i x_i), column G = 64 b + g and rows
// k = RU (4 c + qq) .. RU (4 c + qq) + RU - 1; NB = n_res / 64, QK = 4 * (number of chunks),
// with the columns padded to n_res (a multiple of 256) and the rows to a multiple of 64, the
// pads zero.  A 256-column block of one plane is then four 4 KB runs per chunk.
#include <cmath>

#include "hs_internal.h"
#include "tiles.h"

namespace hsb {

namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void* lds_ptr;

constexpr int kNormRows = 512;  // stacked rows per partial sum of the column norms

// Partial sums of squares over kNormRows rows: part[(op * nkb + kb) * n_res + G] for
// op 0: W, 1: lam W, 2: Y (columns G >= n_pad are zero).
__global__ void __launch_bounds__(256) k_crt_norm_part(const d2* __restrict__ W, const d2* __restrict__ Y,
                                                       const double* __restrict__ lam, int K, int n_pad, int n_res,
                                                       int nkb, double* __restrict__ part) {
  const int G = blockIdx.x * 256 + threadIdx.x;
  if (G >= n_res) return;
  const int kb = blockIdx.y;
  const int k0 = kb * kNormRows, k1 = min(k0 + kNormRows, K);
  double sw = 0.0, sl = 0.0, sy = 0.0;
  if (G < n_pad) {
    for (int k = k0; k < k1; ++k) {
      const d2 w = W[(int64_t)k * n_pad + G];
      const d2 y = Y[(int64_t)k * n_pad + G];
      const double a = w.x * w.x + w.y * w.y;
      const double lk = lam[k];
      sw += a;
      sl += lk * lk * a;
      sy += y.x * y.x + y.y * y.y;
    }
  }
  part[((int64_t)0 * nkb + kb) * n_res + G] = sw;
  part[((int64_t)1 * nkb + kb) * n_res + G] = sl;
  part[((int64_t)2 * nkb + kb) * n_res + G] = sy;
}

// scale[op * n_res + G] = 2^f, the largest power of two with 2^f ||x_G|| + sqrt(2K)/2 <= bound
// (the second term bounds the 2-norm of the rounding errors); 1 for a zero column.  The
// partial sums are added in a fixed order, so the scales are reproducible.
__global__ void __launch_bounds__(256) k_crt_scale(const double* __restrict__ part, int nkb, int n_res, int K,
                                                   double bound, double* __restrict__ scale) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= 3 * n_res) return;
  const int op = i / n_res, G = i - op * n_res;
  double s = 0.0;
  for (int kb = 0; kb < nkb; ++kb) s += part[((int64_t)op * nkb + kb) * n_res + G];
  double sc = 1.0;
  if (s > 0.0) {
    const double t = (bound - 0.5 * sqrt(2.0 * (double)K)) / sqrt(s) * (1.0 - 0x1p-30);
    int e = 0;
    (void)frexp(t, &e);  // t = mant * 2^e, mant in [0.5, 1): 2^(e-1) <= t
    sc = ldexp(1.0, e - 1);
  }
  scale[i] = sc;
}

// v - m * round(v / m), in [-(m-1)/2, (m-1)/2], for an integer-valued double |v| < 2^48 and an
// odd modulus 113 <= m < 256.  The computed v * fl(1/m) is within |v/m| 2^-52 < 2^-10 of v/m,
// while v/m, with m odd, is never closer than 1/(2m) > 2^-9 to a half-integer: the rounded
// quotient is exact, and so are q m and the difference (fma).
__device__ __forceinline__ double smod_d(double v, double m, double inv_m) {
  return fma(-rint(v * inv_m), m, v);
}

// Residue r (an integer in [-(m-1)/2, (m-1)/2], as a double) as the element of kind EK: a signed
// byte (0), or the bits of a bfloat16 (1) or an IEEE half (2), both exact for |r| <= 256.
template <int EK>
__device__ __forceinline__ unsigned residue_bits(double r) {
  if constexpr (EK == 0) return (unsigned)(int)r & 0xffu;
  else if constexpr (EK == 1) return (unsigned)__builtin_bit_cast(unsigned short, (__bf16)(float)r);
  // through int and float (both exact here): a direct double -> half cast is rounded in software
  else return (unsigned)__builtin_bit_cast(unsigned short, (_Float16)(float)(int)r);
}

// One thread per (column G, unit q of RU = 16 (bytes) or 8 (16-bit elements) rows): the 2 n_mod
// residue planes of those rows of X (times lam if use_lam), scaled by scale[G] and rounded.
template <int EK>
__global__ void __launch_bounds__(256) k_crt_residues(CrtConsts cc, const d2* __restrict__ X,
                                                      const double* __restrict__ lam, int use_lam, int K, int n_pad,
                                                      int n_res, int QK, const double* __restrict__ scale,
                                                      u4* __restrict__ out) {
  constexpr int RU = EK == 0 ? 16 : 8;  // rows per 16-byte unit
  constexpr int EB = 16 / RU;           // bytes per element
  const int g = threadIdx.x & 63;
  const int q = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int b = blockIdx.x;
  const int G = b * 64 + g;
  if (q >= QK) return;
  const double sc = scale[G];
  double re[RU], im[RU];
#pragma unroll
  for (int r = 0; r < RU; ++r) {
    const int k = q * RU + r;
    d2 v = d2{0.0, 0.0};
    if (k < K && G < n_pad) {
      v = X[(int64_t)k * n_pad + G];
      if (use_lam) v *= lam[k];
    }
    re[r] = rint(v.x * sc);  // the scale is a power of two: the product is exact
    im[r] = rint(v.y * sc);
  }
  const int NB = n_res / 64;
  const int64_t modstride = (int64_t)2 * NB * QK * 64;
  u4* o = out + ((((int64_t)(q >> 2) * NB + b) * 2) * 4 + (q & 3)) * 64 + g;
  for (int i = 0; i < cc.n_mod; ++i) {
    const double m = (double)cc.m[i], inv_m = 1.0 / m, jm = (double)cc.j[i];
    u4 u0 = u4{0u, 0u, 0u, 0u}, u1 = u4{0u, 0u, 0u, 0u};
#pragma unroll
    for (int r = 0; r < RU; ++r) {
      // c = x_i mod m; x_r + j c (exact: |x_r| < 2^48, |j c| < 2^15) mod m; then
      // x_r - j c = (x_r + j c) - 2 j c from small values (|.| < 2^16)
      const double c = smod_d(im[r], m, inv_m);
      const double p0 = smod_d(fma(jm, c, re[r]), m, inv_m);
      const double p1 = smod_d(fma(-2.0 * jm, c, p0), m, inv_m);
      constexpr int PER = 4 / EB;  // elements per 32-bit word
      u0[r / PER] |= residue_bits<EK>(p0) << (8 * EB * (r % PER));
      u1[r / PER] |= residue_bits<EK>(p1) << (8 * EB * (r % PER));
    }
    o[i * modstride] = u0;
    o[i * modstride + 256] = u1;
  }
}

__device__ __forceinline__ i16v mfma_i8(u4 a, u4 b, i16v c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(i4v, a), __builtin_bit_cast(i4v, b), c, 0, 0, 0);
}

// One 32 x 32 residue MFMA over a unit of K: 32 rows of bytes into int32 sums (EK 0), or 16 rows
// of bfloat16 (1) or half (2) values into FP32 sums, exact for integers below 2^24.
template <int EK>
struct CrtAcc;
template <>
struct CrtAcc<0> {
  typedef i16v T;
  static __device__ __forceinline__ T mma(u4 a, u4 b, T c) { return mfma_i8(a, b, c); }
};
template <>
struct CrtAcc<1> {
  typedef f32x16 T;
  static __device__ __forceinline__ T mma(u4 a, u4 b, T c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
  }
};
template <>
struct CrtAcc<2> {
  typedef f32x16 T;
  static __device__ __forceinline__ T mma(u4 a, u4 b, T c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                  0, 0, 0);
  }
};

// v mod m in [-(m-1)/2, (m-1)/2] for an integer-valued float |v| < 2^24: the quotient from FP32 is
// off by at most one (|v/m| < 2^17.2, relative error 2^-22), q m and v - q m are exact.
__device__ __forceinline__ float smod_f(float v, float m, float inv_m, float h) {
  const float q = rintf(v * inv_m);
  float r = fmaf(-q, m, v);
  r = r > h ? r - m : r;
  r = r < -h ? r + m : r;
  return r;
}

// v mod m in [-(m-1)/2, (m-1)/2] for |v| < 2^30 (the quotient from FP64, one correction).
__device__ __forceinline__ int smod_i(int v, int m, double inv_m, int h) {
  const int q = (int)rint((double)v * inv_m);
  int r = v - q * m;
  if (r > h) r -= m;
  if (r < -h) r += m;
  return r;
}

// Contraction tile: one product (P, Q, or the real product) over a 256 x 256 block of
// (G', G) per workgroup, so each side needs one residue plane: a chunk of the stacked index
// is 16 KB of left and 16 KB of right residues, copied straight into LDS
// (global_load_lds_dwordx4) through a ring of four 32 KB stages, three chunks ahead of its use.
// (Computing P and Q together on a 256 x 128 tile takes the same registers and MFMAs but copies
// 48 KB per chunk: both planes of both sides.)  WAVES = 8: waves of 64 x 128 (2 x 4 blocks of
// 32 x 32, two waves per SIMD); WAVES = 4: waves of 128 x 128 (4 x 4 blocks, one wave per SIMD,
// 2/3 of the LDS reads per MFMA).
constexpr int kCrtStages = 4;
constexpr int kCrtSideUnits = 4 * 4 * 64;                 // 4 blocks of 64 columns x 4 row groups x 64
constexpr int kCrtStageUnits = 2 * kCrtSideUnits;         // left, then right (32 KB)
constexpr int kCrtCopies = kCrtStageUnits / 64;           // 1 KB copies per chunk (32)
constexpr int kCrtWindow = 1024;  // chunks (65536 rows) between reductions of the int32 sums: 2^16 * 120^2 < 2^30
// 16-bit elements: chunks of 32 rows; FP32 sums stay exact integers below 2^24 for 1024 rows
// (2^10 * 120^2 + 120 < 2^24), so they are reduced modulo m every 32 chunks (8-wave layout).
constexpr int kCrtWindow16 = 32;
// Byte form: chunks whose sums stay exact with no reduction at all: 2^17 rows * 120^2 < 2^31.
// Reducing 256 accumulators held in AGPRs inside the loop makes the 4-wave layout spill, so it
// has no reduction, runs only up to this many chunks and the 8-wave layout takes longer
// stacked widths (and the 16-bit forms, which reduce every 32 chunks).
constexpr int kCrtNoReduce = 2048;

// s_waitcnt immediates (gfx9 encoding): vector-memory count N, the other counters not waited on.
constexpr int vmcnt_only(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// Workgroup w: (modulus, product) = w / num_tiles, product fastest (P then Q; the real form has
// one), 256 x 256 block w % num_tiles of the upper triangle (XCD-contiguous numbering, so the
// blocks an XCD runs together belong to one modulus and product and to a compact patch of the
// triangle).  P multiplies the left plane 1 (x_r - j x_i) by the right plane 0 (y_r + j y_i), Q
// the left plane 0 by the right plane 1.  The real form wants Re = (P + Q) / 2 only: it adds both
// products into one sum, running through 2 x (chunks) stages, each chunk once with the planes
// of P and once with those of Q.
// res: residues in [-(m-1)/2, (m-1)/2] as signed bytes, [n_mod][nprod][n_res][n_res] (the real
// form: of Re), written for row <= col < n (the 4-wave layout writes the whole of each 256 x 256
// block it computes, inside the plane).
template <int EK, int WAVES, bool REAL>
__global__ void __launch_bounds__(WAVES * 64, 1) k_hs_crt(const u4* __restrict__ L, const u4* __restrict__ R,
                                                          CrtConsts cc, int QK, int n, int NB, int nbs,
                                                          int num_tiles, int num_wg, int gr, int8_t* __restrict__ res,
                                                          int64_t ld) {
  constexpr int NPROD = REAL ? 1 : 2;
  constexpr int WRN = WAVES / 2;           // wave rows
  constexpr int RB = 8 / WRN;              // 32-row blocks per wave (2 or 4); 4 column blocks
  constexpr int NPW = kCrtCopies / WAVES;  // copies per wave and chunk (4 or 8)
  constexpr int NMF = 2 * RB * 4;          // MFMAs per wave and chunk (16 or 32)
  static_assert(NPW <= NMF / 2, "one copy per MFMA pair of the chunk");
  __shared__ u4 lds[kCrtStages][kCrtStageUnits];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int x = blockIdx.x % kXcds;
  int start, len;
  xcd_range(x, num_wg, start, len);
  const int w = start + blockIdx.x / kXcds;
  const int mp = w / num_tiles;
  const int mod = mp / NPROD, prod = mp - mod * NPROD;
  int bi, bj;
  if (gr > 0) grouped_decode(w - mp * num_tiles, nbs, gr, bi, bj);
  else tri_decode(w - mp * num_tiles, nbs, bi, bj);
  const int row0 = bi * 256, col0 = bj * 256;
  if (col0 >= n) return;
  const int planeL = 1 - prod, planeR = prod;  // the real form starts with P's planes
  const int64_t modstride = (int64_t)2 * NB * QK * 64, cstride = (int64_t)NB * 512;  // units
  const u4* Lm = L + mod * modstride;
  const u4* Rm = R + mod * modstride;

  const u4* src[NPW];
  int dst[NPW], dlt[NPW];
#pragma unroll
  for (int i = 0; i < NPW; ++i) {
    const int j = wave + WAVES * i;  // copy j: side j / 16, block (j / 4) % 4, row group j % 4
    const int side = j >> 4, b = (j >> 2) & 3, qq = j & 3;
    const u4* base = side ? Rm : Lm;
    const int b0 = side ? (col0 >> 6) : (row0 >> 6);
    src[i] = base + (((b0 + b) * 2 + (side ? planeR : planeL)) * 4 + qq) * 64;
    dst[i] = side * kCrtSideUnits + (b * 4 + qq) * 64;
    dlt[i] = side ? 256 : -256;  // real form, Q's stage: the other plane of each side
  }
  // stage v: chunk v (complex), or chunk v / 2 with P's (v even) or Q's (v odd) planes (real)
  auto at = [&](int i, int v) -> const u4* {
    if constexpr (REAL) return src[i] + (v >> 1) * cstride + (v & 1) * dlt[i];
    else return src[i] + v * cstride;
  };
  auto issue = [&](int v, int buf) {
#pragma unroll
    for (int i = 0; i < NPW; ++i)
      __builtin_amdgcn_global_load_lds((const void*)(at(i, v) + lane), (lds_ptr)(&lds[buf][dst[i]]), 16, 0, 0);
  };

  typedef CrtAcc<EK> Mma;
  typename Mma::T acc[RB][4];
#pragma unroll
  for (int a = 0; a < RB; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0;

  const int m = cc.m[mod], hm = (m - 1) / 2;
  const double inv_m = 1.0 / (double)m;
  const float mf = (float)m, inv_mf = 1.0f / mf, hmf = (float)hm;
  auto reduce = [&]() {
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          if constexpr (EK == 0) acc[a][b][r] = smod_i(acc[a][b][r], m, inv_m, hm);
          else acc[a][b][r] = smod_f(acc[a][b][r], mf, inv_mf, hmf);
        }
  };

  const int qh = lane >> 5, g32 = lane & 31;
  // A operand of row block rb (rows 32 (RB wr + rb) of the block) at step s (rows 32 s .. 32 s + 31
  // of the chunk): left unit ((RB wr + rb) / 2 * 4 + 2 s + qh) * 64 + ((RB wr + rb) & 1) * 32 + g32.
  // B operand of column block cb (columns 32 (4 wc + cb)): right unit
  // kCrtSideUnits + ((4 wc + cb) / 2 * 4 + 2 s + qh) * 64 + (cb & 1) * 32 + g32.
  const int la = qh * 64 + g32;
  const int ra = kCrtSideUnits + (2 * wc * 4 + qh) * 64 + g32;
  const int nchunks = (QK >> 2) * (REAL ? 2 : 1);  // stages
#pragma unroll
  for (int i = 0; i < kCrtStages - 1; ++i)
    if (i < nchunks) issue(i, i);
  for (int c = 0; c < nchunks; ++c) {
    // this wave's copies of chunk c are done once at most those of the chunks after it
    // (up to kCrtStages - 2 of them) are pending
    const int pend = min(kCrtStages - 2, nchunks - 1 - c);
    if (pend >= 2) __builtin_amdgcn_s_waitcnt(vmcnt_only(2 * NPW));
    else if (pend == 1) __builtin_amdgcn_s_waitcnt(vmcnt_only(NPW));
    else __builtin_amdgcn_s_waitcnt(vmcnt_only(0));
    // Every wave's copies of chunk c are in LDS past this barrier, and stage (c - 1) % 4 is
    // free (its reads, of chunk c - 1, fed MFMAs before the barrier).  A plain s_barrier: the
    // release fence of __syncthreads would wait for the copies still in flight as well.
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    // The copies of chunk c + 3 go out one after each pair of MFMAs (scheduling fences keep
    // them there): issued together after the barrier they hold up the MFMAs behind them.
    const bool more = c + kCrtStages - 1 < nchunks;
    const int nbuf = (c + kCrtStages - 1) % kCrtStages;
    const u4* B = lds[c % kCrtStages];
    int ci = 0;
    u4 a[2][RB], b[2][4];
    auto read_a = [&](int s, int t0, int t1) {
#pragma unroll
      for (int t = t0; t < t1; ++t) {
        const int rbb = RB * wr + t;
        a[s][t] = B[la + ((rbb >> 1) * 4 + 2 * s) * 64 + (rbb & 1) * 32];
      }
    };
    auto read_b = [&](int s) {
#pragma unroll
      for (int t = 0; t < 4; ++t) b[s][t] = B[ra + ((t >> 1) * 4 + 2 * s) * 64 + (t & 1) * 32];
    };
    // With one wave per SIMD (4 waves) the chunk's first MFMA waits only for the operands of
    // row block 0 (5 reads), and the other row blocks' are read right after it; with two waves
    // per SIMD the other wave covers that wait, and all 8 are read at once.
    read_a(0, 0, WAVES == 4 ? 1 : RB);
    read_b(0);
    if constexpr (WAVES == 4) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          acc[rb][cb] = Mma::mma(a[s][rb], b[s][cb], acc[rb][cb]);
          if constexpr (WAVES == 4) {
            if (s == 0 && rb == 0 && cb == 0) {
              read_a(0, 1, RB);
              __builtin_amdgcn_sched_barrier(0);
            }
          }
          if ((cb & 1) && more && ci < NPW)
            __builtin_amdgcn_global_load_lds((const void*)(at(ci, c + kCrtStages - 1) + lane),
                                             (lds_ptr)(&lds[nbuf][dst[ci]]), 16, 0, 0);
          if (cb & 1) {
            ++ci;
            __builtin_amdgcn_sched_barrier(0);
          }
          // the second step's operands are read halfway through the first step's MFMAs, so
          // their LDS latency is hidden behind the rest of them
          if (s == 0 && rb * 4 + cb == 2 * RB - 1) {
            read_a(1, 0, RB);
            read_b(1);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
    }
    // the 4-wave byte form runs only where no reduction is needed (at most kCrtNoReduce stages)
    if constexpr (EK != 0) {
      if ((c + 1) % kCrtWindow16 == 0) reduce();
    } else if constexpr (WAVES == 8) {
      if ((c + 1) % kCrtWindow == 0) reduce();
    }
  }

  // Residues of the product (the real form: of (P + Q) / 2).  Output element r of a 32 x 32 block:
  // row 8 (r / 4) + 4 qh + r % 4, column g32.
  if constexpr (WAVES == 4) {
    // Each sum is an exact integer below 2^31 in magnitude, reduced in FP64 as the residues of
    // the operands are.  Every element of the block is written: the block lies inside the
    // n_res x n_res plane, its rows and columns past n hold products of zero pads, and the
    // recombination reads row <= col < n only.  The wave's base is made visibly uniform, so the
    // per-element offsets are scalar arithmetic.
    const double md = (double)m;
    const double inv2 = REAL ? (double)cc.inv2[mod] : 0.0;
    auto residue = [&](double v) -> int8_t {
      double r = smod_d(v, md, inv_m);
      if constexpr (REAL) r = smod_d(r * inv2, md, inv_m);  // (P + Q) / 2
      return (int8_t)(int)r;
    };
    const uint64_t wb = (uint64_t)(res + (int64_t)(mod * NPROD + prod) * ld * ld +
                                   (int64_t)(row0 + wr * 32 * RB) * ld + col0 + wc * 128);
    // (readfirstlane returns a signed int: each half goes through unsigned, or the low one would
    // sign-extend into the high word)
    const unsigned wb_hi = (unsigned)__builtin_amdgcn_readfirstlane((unsigned)(wb >> 32));
    const unsigned wb_lo = (unsigned)__builtin_amdgcn_readfirstlane((unsigned)wb);
    typedef __attribute__((address_space(1))) int8_t gbyte;
    gbyte* const ow = (gbyte*)(((uint64_t)wb_hi << 32) | (uint64_t)wb_lo);
    const unsigned lane_off = (unsigned)(4 * qh) * (unsigned)ld + (unsigned)g32;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          ow[(int64_t)(rb * 32 + 8 * (r >> 2) + (r & 3)) * ld + cb * 32 + lane_off] = residue((double)acc[rb][cb][r]);
  } else {
    // (the 8-wave layout keeps per-element bounds: written this way, the 16-bit forms measured
    // 5 % faster than with the 4-wave epilogue)
    const int inv2 = REAL ? cc.inv2[mod] : 0;
    int rbase = row0 + wr * 32 * RB + 4 * qh, cbase = col0 + wc * 128 + g32;
    asm volatile("" : "+v"(rbase), "+v"(cbase));
    int8_t* out = res + (int64_t)(mod * NPROD + prod) * ld * ld;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = rbase + rb * 32 + 8 * (r >> 2) + (r & 3);
          const int col = cbase + cb * 32;
          if (row < n && col < n && col >= row) {
            int v = smod_i((int)acc[rb][cb][r], m, inv_m, hm);  // 16-bit forms: an exact integer < 2^24
            if constexpr (REAL) v = smod_i(v * inv2, m, inv_m, hm);  // (P + Q) / 2
            out[(int64_t)row * ld + col] = (int8_t)v;
          }
        }
  }
}

// Recovery of each upper-triangle entry from its residues: value = M * frac(sum_i r_i y_i / m_i),
// times 2^-(f_row + f_col), with r_i the residue of the real form's one product, or of
// Re = (P + Q) / 2 and Im = (P - Q) / (2 j) (mod m).  The fraction depends on r_i only modulo m_i,
// so the complex form takes r_i = P + Q and P - Q as they are (|r_i| <= 240) against the weights
// 2^{-1} y_i and (2 j)^{-1} y_i (mod m_i), with no reduction.  sum r_i h_i is exact (h_i on a
// 2^-42 grid with |r_i| < 2^7, or on a 2^-41 grid with |r_i| < 2^8; n <= 13 terms, so the sums
// stay below 2^12), the rounding to the nearest integer is exact and the fraction keeps FP64
// precision.  One thread per four consecutive columns of a row (4-byte
// loads of the residues; the rows are n_res bytes long, so the four are always in the row).
template <bool REAL>
__global__ void __launch_bounds__(256) k_crt_combine(CrtConsts cc, const int8_t* __restrict__ res, int64_t ld,
                                                     const double* __restrict__ scL, const double* __restrict__ scR,
                                                     int n, void* __restrict__ Cv) {
  const int row = blockIdx.y;
  const int col0 = (blockIdx.x * 256 + threadIdx.x) * 4;
  if (col0 >= n || col0 + 3 < row) return;
  const int64_t mstride = ld * ld, e = (int64_t)row * ld + col0;
  double hr[4] = {0.0, 0.0, 0.0, 0.0}, lr[4] = {0.0, 0.0, 0.0, 0.0};
  double hi[4] = {0.0, 0.0, 0.0, 0.0}, li[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < cc.n_mod; ++i) {
    if constexpr (REAL) {
      const double h = cc.h[i], l = cc.l[i];
      const unsigned v = *(const unsigned*)(res + i * mstride + e);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double r = (double)(int8_t)(v >> (8 * u));
        hr[u] += r * h;
        lr[u] += r * l;
      }
    } else {
      const unsigned vp = *(const unsigned*)(res + (2 * i) * mstride + e);
      const unsigned vq = *(const unsigned*)(res + (2 * i + 1) * mstride + e);
      const double h_re = cc.h_re[i], l_re = cc.l_re[i], h_im = cc.h_im[i], l_im = cc.l_im[i];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int p = (int8_t)(vp >> (8 * u)), q = (int8_t)(vq >> (8 * u));
        const double r = (double)(p + q), t = (double)(p - q);
        hr[u] += r * h_re;
        lr[u] += r * l_re;
        hi[u] += t * h_im;
        li[u] += t * l_im;
      }
    }
  }
  const double sl = cc.M / scL[row];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int col = col0 + u;
    if (col < n && col >= row) {
      const double sc = sl / scR[col];
      const double fr = (hr[u] - rint(hr[u])) + lr[u];
      if constexpr (REAL) {
        ((double*)Cv)[(int64_t)row * n + col] = fr * sc;
      } else {
        const double fi = (hi[u] - rint(hi[u])) + li[u];
        ((d2*)Cv)[(int64_t)row * n + col] = d2{fr * sc, fi * sc};
      }
    }
  }
}

}  // namespace

namespace {
int inverse_mod(int a, int m) {  // a^{-1} mod m for gcd(a, m) = 1, m < 256
  a %= m;
  if (a < 0) a += m;
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 0;
}
}  // namespace

// The n_mod largest moduli below 256 that are powers of distinct primes p = 1 (mod 4):
// 241, 233, 229, 197, 193, 181, 173, 169 = 13^2, 157, 149, 137, 125 = 5^3, 113, 109, ...
bool crt_make_consts(int n_mod, CrtConsts* cc) {
  if (n_mod < kCrtMinModuli || n_mod > kCrtMaxModuli || !cc) return false;
  *cc = CrtConsts{};
  cc->n_mod = n_mod;
  int used[64], n_used = 0, k = 0;
  for (int m = 255; m >= 5 && k < n_mod; --m) {
    int p = 2;
    while (m % p) ++p;  // smallest prime factor
    int r = m;
    while (r % p == 0) r /= p;
    if (r != 1 || p % 4 != 1) continue;
    bool dup = false;
    for (int i = 0; i < n_used; ++i) dup = dup || used[i] == p;
    if (dup) continue;
    used[n_used++] = p;
    int j = 1;
    while ((j * j + 1) % m) ++j;
    cc->m[k] = m;
    cc->j[k] = j;
    cc->inv2[k] = inverse_mod(2, m);
    cc->inv2j[k] = inverse_mod(2 * j, m);
    ++k;
  }
  if (k < n_mod) return false;
  double M = 1.0;
  for (int i = 0; i < n_mod; ++i) M *= (double)cc->m[i];
  for (int i = 0; i < n_mod; ++i) {
    const int mi = cc->m[i];
    int c = 1;  // (M / m_i) mod m_i
    for (int t = 0; t < n_mod; ++t)
      if (t != i) c = c * (cc->m[t] % mi) % mi;
    const int y = inverse_mod(c, mi);
    // w / m_i = h + l with h on a 2^-bits grid; w - h m_i is exact (h has at most 42 fractional
    // bits, m_i 8 bits)
    auto split = [mi](int w, int bits, double& h, double& l) {
      h = std::ldexp(std::rint(std::ldexp((double)w / mi, bits)), -bits);
      l = ((double)w - h * mi) / mi;
    };
    split(y, 42, cc->h[i], cc->l[i]);
    split(cc->inv2[i] * y % mi, 41, cc->h_re[i], cc->l_re[i]);
    split(cc->inv2j[i] * y % mi, 41, cc->h_im[i], cc->l_im[i]);
  }
  cc->M = M;
  cc->bound = std::sqrt(0.5 * M * (1.0 - 0x1p-10));
  return true;
}

int crt_norm_blocks(int K) { return (K + kNormRows - 1) / kNormRows; }

int crt_tiles(int n_res) {
  const int nbs = n_res / 256;
  return nbs * (nbs + 1) / 2;
}

hipError_t launch_crt_scales(const double2* W, const double2* Y, const double* lam, int K, int n_pad, int n_res,
                             const CrtConsts& cc, double* part, double* scale, hipStream_t s) {
  const int nkb = crt_norm_blocks(K);
  hipLaunchKernelGGL(k_crt_norm_part, dim3(n_res / 256, nkb), dim3(256), 0, s, (const d2*)W, (const d2*)Y, lam, K,
                     n_pad, n_res, nkb, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_crt_scale, dim3((3 * n_res + 255) / 256), dim3(256), 0, s, (const double*)part, nkb, n_res, K,
                     cc.bound, scale);
  return hipGetLastError();
}

hipError_t launch_crt_residues(const CrtConsts& cc, int ek, const double2* X, const double* lam, int use_lam, int K,
                               int n_pad, int n_res, int QK, const double* scale, void* out, hipStream_t s) {
  dim3 grid(n_res / 64, (QK + 3) / 4);
  if (ek == 0)
    hipLaunchKernelGGL(k_crt_residues<0>, grid, dim3(256), 0, s, cc, (const d2*)X, lam, use_lam, K, n_pad, n_res, QK,
                       scale, (u4*)out);
  else if (ek == 1)
    hipLaunchKernelGGL(k_crt_residues<1>, grid, dim3(256), 0, s, cc, (const d2*)X, lam, use_lam, K, n_pad, n_res, QK,
                       scale, (u4*)out);
  else
    hipLaunchKernelGGL(k_crt_residues<2>, grid, dim3(256), 0, s, cc, (const d2*)X, lam, use_lam, K, n_pad, n_res, QK,
                       scale, (u4*)out);
  return hipGetLastError();
}

namespace {
template <int EK>
void launch_hs_crt_k(bool real, bool four, dim3 grid, const u4* l, const u4* r, const CrtConsts& cc, int QK, int n,
                     int NB, int nbs, int num_tiles, int num_wg, int gr, int8_t* o, int64_t ld, hipStream_t s) {
  if constexpr (EK == 0) {
    if (four) {
      if (real)
        hipLaunchKernelGGL((k_hs_crt<EK, 4, true>), grid, dim3(256), 0, s, l, r, cc, QK, n, NB, nbs, num_tiles,
                           num_wg, gr, o, ld);
      else
        hipLaunchKernelGGL((k_hs_crt<EK, 4, false>), grid, dim3(256), 0, s, l, r, cc, QK, n, NB, nbs, num_tiles,
                           num_wg, gr, o, ld);
      return;
    }
  }
  {
    if (real)
      hipLaunchKernelGGL((k_hs_crt<EK, 8, true>), grid, dim3(512), 0, s, l, r, cc, QK, n, NB, nbs, num_tiles, num_wg,
                         gr, o, ld);
    else
      hipLaunchKernelGGL((k_hs_crt<EK, 8, false>), grid, dim3(512), 0, s, l, r, cc, QK, n, NB, nbs, num_tiles, num_wg,
                         gr, o, ld);
  }
}
}  // namespace

hipError_t launch_hs_crt(const CrtConsts& cc, int ek, bool real, const void* L, const void* R, int QK, int n,
                         int n_res, int gr, int waves, void* res, hipStream_t s) {
  const int nbs = n_res / 256;
  const int num_tiles = crt_tiles(n_res);
  const int num_wg = num_tiles * cc.n_mod * (real ? 1 : 2);
  const int NB = n_res / 64;
  const dim3 grid(num_wg);
  const u4 *l = (const u4*)L, *r = (const u4*)R;
  int8_t* o = (int8_t*)res;
  const int64_t ld = n_res;
  // The byte form's 4-wave layout has no reduction of its sums: it runs up to kCrtNoReduce stages.
  // The 16-bit forms reduce their FP32 sums every 32 chunks, which the 4-wave layout, its 256
  // sums in AGPRs, could only do by spilling inside the loop: they run the 8-wave layout.
  const bool four = waves == 4 && ek == 0 && QK / 4 * (real ? 2 : 1) <= kCrtNoReduce;
  if (ek == 0) launch_hs_crt_k<0>(real, four, grid, l, r, cc, QK, n, NB, nbs, num_tiles, num_wg, gr, o, ld, s);
  else if (ek == 1) launch_hs_crt_k<1>(real, four, grid, l, r, cc, QK, n, NB, nbs, num_tiles, num_wg, gr, o, ld, s);
  else launch_hs_crt_k<2>(real, four, grid, l, r, cc, QK, n, NB, nbs, num_tiles, num_wg, gr, o, ld, s);
  return hipGetLastError();
}

hipError_t launch_crt_combine(const CrtConsts& cc, bool real, const void* res, int n_res, const double* scL,
                              const double* scR, int n, void* C, hipStream_t s) {
  dim3 grid((n + 1023) / 1024, n);
  const int8_t* r = (const int8_t*)res;
  if (real)
    hipLaunchKernelGGL((k_crt_combine<true>), grid, dim3(256), 0, s, cc, r, (int64_t)n_res, scL, scR, n, C);
  else
    hipLaunchKernelGGL((k_crt_combine<false>), grid, dim3(256), 0, s, cc, r, (int64_t)n_res, scL, scR, n, C);
  return hipGetLastError();
}

}  // namespace hsb
