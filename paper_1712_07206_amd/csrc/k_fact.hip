// Type-factored ("compressed") H and S (the compression of A and B that
// Sec. 7 names as future work, worked out for the stacked form of Eqs. 6-7).
//
// Every coefficient of atom a (type t) is its type's coefficient at the origin
// times the atom's structure phase: W_a[k][G] = E_a(G) W0_t[k][G] with
// E_a(G) = e^{i K_G . tau_a} and k = (A|B, L).  Because T and the radial data are
// per type, the atom sum of Eqs. 4-5 factors entry by entry:
//
//   H[G'][G] = sum_t P_t[G'][G] (W0_t^H Y0_t)[G'][G],        Y0_t = T_t W0_t
//   S[G'][G] = sum_t P_t[G'][G] (W0_t^H Lam_t W0_t)[G'][G]
//   P_t[G'][G] = sum_{a in t} conj(E_a(G')) E_a(G)
//
// so the contraction width per entry drops from 4 N_atoms N_L (the stacked
// form) to sum_t (N_t + 4 N_L), plus one complex product per type.
//
// One workgroup per 64 x 64 tile of the upper triangle, 8 waves of 32 x 16
// (two waves per SIMD).  Per type the tile first contracts the phases (K = N_t
// rows of E), then W0_t against Y0_t and Lam_t W0_t together (K = 2 N_L, the
// left operand shared), and folds M_H * P and M_S * P into the running H and S
// tiles in registers; nothing but the final tile goes back to HBM.  All
// contractions are complex FP64 on v_mfma_f64_16x16x4f64; rows are copied 16 at
// a time straight into double-buffered LDS (global_load_lds, no staging
// registers), the next chunk's copies issued while the current one is
// contracted; the next chunk may belong to the next phase or type.
#include "hs_internal.h"
#include "tiles.h"

namespace hsb {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int FM = 64, FK = 16, FNT = 512;
#define MFMA(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)

// E[a][G] = e^{i K_G . tau_a} for every atom; one thread per G.
__global__ void __launch_bounds__(256) k_phases(int n_atoms, int n_pad, const double* __restrict__ kv,
                                                const double* __restrict__ tau, double2* __restrict__ E) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= n_pad) return;
  const double kx = kv[4 * (int64_t)G + 0], ky = kv[4 * (int64_t)G + 1], kz = kv[4 * (int64_t)G + 2];
  for (int a = blockIdx.y; a < n_atoms; a += gridDim.y) {
    double s, c;
    sincos(kx * tau[3 * a + 0] + ky * tau[3 * a + 1] + kz * tau[3 * a + 2], &s, &c);
    E[(int64_t)a * n_pad + G] = make_double2(c, s);
  }
}

// Row metadata of the factored layout (rows type by type: E block, then W0 block,
// each padded to 16): lamx[r] (1 on E rows and A rows, ||udot_l||^2 on B rows,
// 0 on pad rows) and kind[] of each 16-row chunk.
__global__ void __launch_bounds__(256) k_fact_rows(CellArgs c, const TypeConsts* __restrict__ consts, int rows,
                                                   double* __restrict__ lamx, int* __restrict__ kind) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int K = 2 * c.n_l, Mp = (K + FK - 1) / FK * FK;
  int base = 0, t = 0, nt = 0, Ep = 0;
  for (t = 0; t < c.n_types; ++t) {
    nt = c.type_start[t + 1] - c.type_start[t];
    if (nt == 0) continue;
    Ep = (nt + FK - 1) / FK * FK;
    if (r < base + Ep + Mp) break;
    base += Ep + Mp;
  }
  const int rr = r - base;  // base is a multiple of 16
  double lam;
  int kd;
  int valid;  // data rows in this row's chunk
  if (rr < Ep) {
    lam = rr < nt ? 1.0 : 0.0;
    kd = rr / FK == Ep / FK - 1 ? 3 : 0;
    valid = min(FK, nt - rr / FK * FK);
  } else {
    const int m = rr - Ep;
    if (m < c.n_l) {
      lam = 1.0;
    } else if (m < K) {
      const int L = m - c.n_l;
      int l = 0;
      while ((l + 1) * (l + 1) <= L) ++l;
      lam = consts->udot2[t][l];
    } else {
      lam = 0.0;
    }
    kd = m / FK == Mp / FK - 1 ? 2 : 1;
    valid = min(FK, K - m / FK * FK);
  }
  kd |= ((valid + 3) / 4 - 1) << 2;
  lamx[r] = lam;
  if (rr % FK == 0) kind[r / FK] = kd;
}

// XL[r][G] = lam[r] X[r][G]; one thread per G, rows over blockIdx.y.
__global__ void __launch_bounds__(256) k_scale_rows(const double2* __restrict__ X, const double* __restrict__ lam,
                                                    int rows, int n_pad, double2* __restrict__ XL) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= n_pad) return;
  for (int r = blockIdx.y; r < rows; r += gridDim.y) {
    const double2 v = X[(int64_t)r * n_pad + G];
    XL[(int64_t)r * n_pad + G] = make_double2(lam[r] * v.x, lam[r] * v.y);
  }
}

typedef __attribute__((address_space(3))) void* lds_ptr;

// Rows of X, XL and Yx come type by type: the type's E rows, then its W0 rows,
// each block padded with zero rows to a multiple of 16, so every 16-row chunk is
// one kind: kind[c] & 3 = 0 (phases), 3 (the type's last phase chunk), 1 (W0 rows),
// 2 (the type's last W0 chunk, after which M * P is folded into H and S); kind[c] >> 2
// is the number of 4-row steps of the chunk that hold data rows, minus one.
// XL = lam X (lam = 1 on phase rows, ||udot_l||^2 on B rows) and Yx is zero on
// phase rows, so a phase chunk adds E^H E to the S slot and nothing to the H slot.
// The slots sum conj(a) b in the three-product (3M) form, P1 = a_r b_r, P2 = a_i b_i,
// P3 = (a_r - a_i)(b_r + b_i), and are turned into Re = P1 + P2, Im = P3 - P1 + P2
// where a slot is captured (P_t) or folded: 3 MFMAs per complex multiply-add.
__global__ void __launch_bounds__(FNT, 1) k_hs_fact(const d2* __restrict__ X, const d2* __restrict__ XL,
                                                    const d2* __restrict__ Yx, const int* __restrict__ kind,
                                                    int nch, int n, int n_pad, int nb, int num_wg, int gr,
                                                    d2* __restrict__ H, d2* __restrict__ S, int64_t ldh) {
  // per buffer: L (16 rows x 64 at G'), R (16 x 64 of XL at G), Y (16 x 64 of Yx at G)
  __shared__ d2 lds[2][3 * FK * FM];
  const int x = blockIdx.x % kXcds;
  int start, len;
  xcd_range(x, num_wg, start, len);
  const int w = start + blockIdx.x / kXcds;
  int bi, bj;
  if (gr > 0) grouped_decode(w, nb, gr, bi, bj);
  else tri_decode(w, nb, bi, bj);
  const int row0 = bi * FM, col0 = bj * FM;
  if (col0 >= n) return;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 2, wc = wave & 3;  // rows wr*32 (two 16-row blocks), columns wc*16

  // staging straight into LDS: 48 row copies of 1 KB per chunk, wave w takes j = w + 8 i;
  // copy j: array j/16 (X at G', XL at G, Yx at G), row j%16
  const d2* src0[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const int j = wave + 8 * i;
    const int arr = j >> 4, r = j & 15;
    const d2* base = arr == 0 ? X + row0 : (arr == 1 ? XL + col0 : Yx + col0);
    src0[i] = base + (int64_t)r * n_pad;
  }
  auto issue = [&](int c, int buf) {
#pragma unroll
    for (int i = 0; i < 6; ++i)
      __builtin_amdgcn_global_load_lds((const void*)(src0[i] + (int64_t)c * FK * n_pad + lane),
                                       (lds_ptr)(&lds[buf][(wave + 8 * i) * FM]), 16, 0, 0);
  };

  d4 pR[2], pI[2], mh1[2], mh2[2], mh3[2], ms1[2], ms2[2], ms3[2], hR[2], hI[2], sR[2], sI[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    pR[i] = pI[i] = d4{0.0, 0.0, 0.0, 0.0};
    mh1[i] = mh2[i] = mh3[i] = ms1[i] = ms2[i] = ms3[i] = d4{0.0, 0.0, 0.0, 0.0};
    hR[i] = hI[i] = sR[i] = sI[i] = d4{0.0, 0.0, 0.0, 0.0};
  }

  issue(0, 0);
  for (int c = 0; c < nch; ++c) {
    const int b = c & 1;
    const int kc = kind[c];         // uniform
    const int kd = kc & 3, nks = (kc >> 2) + 1;
    const bool hslot = kd == 1 || kd == 2;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of chunk c have landed
    __syncthreads();                // everyone's have, and buffer b^1 is free
    // the next chunk's copies go out before step ki, half-way through a full chunk: issued
    // right after the barrier their LDS writes meet the chunk's first reads (measured:
    // 3.6 % slower); ki < nks, so the early exit below never skips them
    const int ki = nks > 2 ? 2 : nks - 1;
    const d2* L = lds[b];
    const d2* R = lds[b] + FK * FM;
    const d2* Yl = lds[b] + 2 * FK * FM;
    // every chunk adds X^H XL to the S slot (P_t on phase chunks); W0 chunks also add
    // X^H Yx to the H slot.  Only the 4-row steps that hold data rows are run.
#pragma unroll
    for (int ks = 0; ks < FK / 4; ++ks) {
      if (ks == ki && c + 1 < nch) issue(c + 1, b ^ 1);
      if (ks >= nks) break;
      const int kk = ks * 4 + (lane >> 4);
      double ar[2], ai[2], ad[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const d2 a = L[kk * FM + wr * 32 + i * 16 + (lane & 15)];
        ar[i] = a.x; ai[i] = a.y; ad[i] = a.x - a.y;
      }
      const d2 yv = Yl[kk * FM + wc * 16 + (lane & 15)];
      const d2 wv = R[kk * FM + wc * 16 + (lane & 15)];
      const double ws = wv.x + wv.y, ys = yv.x + yv.y;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ms1[i] = MFMA(ar[i], wv.x, ms1[i]);
        ms2[i] = MFMA(ai[i], wv.y, ms2[i]);
        ms3[i] = MFMA(ad[i], ws, ms3[i]);
      }
      if (hslot) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          mh1[i] = MFMA(ar[i], yv.x, mh1[i]);
          mh2[i] = MFMA(ai[i], yv.y, mh2[i]);
          mh3[i] = MFMA(ad[i], ys, mh3[i]);
        }
      }
    }
    if (kd == 3) {  // the type's last phase chunk: the S slot holds P_t
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        pR[i] = ms1[i] + ms2[i];
        pI[i] = ms3[i] - ms1[i] + ms2[i];
        ms1[i] = ms2[i] = ms3[i] = d4{0.0, 0.0, 0.0, 0.0};
      }
    } else if (kd == 2) {  // the type's last W0 chunk: fold M * P into H and S
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const d4 mhR = mh1[i] + mh2[i], mhI = mh3[i] - mh1[i] + mh2[i];
        const d4 msR = ms1[i] + ms2[i], msI = ms3[i] - ms1[i] + ms2[i];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double p_r = pR[i][q], p_i = pI[i][q];
          hR[i][q] += mhR[q] * p_r - mhI[q] * p_i;
          hI[i][q] += mhR[q] * p_i + mhI[q] * p_r;
          sR[i][q] += msR[q] * p_r - msI[q] * p_i;
          sI[i][q] += msR[q] * p_i + msI[q] * p_r;
        }
        mh1[i] = mh2[i] = mh3[i] = ms1[i] = ms2[i] = ms3[i] = d4{0.0, 0.0, 0.0, 0.0};
      }
    }
  }

  // D layout of the 16x16 f64 MFMA: lane l, element q -> row l/16 + 4q, column l%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = row0 + wr * 32 + i * 16 + (lane >> 4) + 4 * q;
      const int col = col0 + wc * 16 + (lane & 15);
      if (row < n && col < n && col >= row) {
        const int64_t o = (int64_t)row * ldh + col;
        H[o] = d2{hR[i][q], hI[i][q]};
        S[o] = d2{sR[i][q], sI[i][q]};
      }
    }
}

}  // namespace

int fact_tiles(int n_pad) {
  const int nb = n_pad / FM;
  return nb * (nb + 1) / 2;
}

hipError_t launch_phases(int n_atoms, int n_pad, const double* kv, const double* tau, double2* E, hipStream_t s) {
  dim3 grid((n_pad + 255) / 256, n_atoms < 64 ? n_atoms : 64);
  hipLaunchKernelGGL(k_phases, grid, dim3(256), 0, s, n_atoms, n_pad, kv, tau, E);
  return hipGetLastError();
}

hipError_t launch_fact_rows(const CellArgs& c, const TypeConsts* consts, int rows, double* lamx, int* kind,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_fact_rows, dim3((rows + 255) / 256), dim3(256), 0, s, c, consts, rows, lamx, kind);
  return hipGetLastError();
}

hipError_t launch_scale_rows(const double2* X, const double* lam, int rows, int n_pad, double2* XL, hipStream_t s) {
  dim3 grid((n_pad + 255) / 256, rows < 256 ? rows : 256);
  hipLaunchKernelGGL(k_scale_rows, grid, dim3(256), 0, s, X, lam, rows, n_pad, XL);
  return hipGetLastError();
}

hipError_t launch_hs_fact(const double2* X, const double2* XL, const double2* Yx, const int* kind, int nch, int n,
                          int n_pad, int gr, double2* H, double2* S, int64_t ldh, hipStream_t s) {
  const int nb = n_pad / FM;
  const int num_wg = fact_tiles(n_pad);
  hipLaunchKernelGGL(k_hs_fact, dim3(num_wg), dim3(FNT), 0, s, (const d2*)X, (const d2*)XL, (const d2*)Yx, kind, nch,
                     n, n_pad, nb, num_wg, gr, (d2*)H, (d2*)S, ldh);
  return hipGetLastError();
}

}  // namespace hsb
