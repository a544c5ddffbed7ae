// Matching coefficients of the LAPW basis (Eq. 2, matched in value and slope
// at the muffin-tin radius, Sec. 2.1).
//
//   k_tables   : per G, K = B(G + k), |K|, the angular factor
//                pre * i^l conj(Y_lm(K_hat)) for every L, and per type the
//                radial matching pair (a_l, b_l).  Small and compute-light.
//   k_assemble : the HBM-write-bound product
//                W[atom][A|B][L][G] = e^{iK_G.tau_atom} * ang[L][G] * (a|b)_{t,l}(G),
//                one thread per G (coalesced 16-byte stores along G) and a
//                group of eight atoms, so each angular factor is read once
//                per eight atoms.
//   k_lambda   : the overlap weight of each stacked row.
#include "hs_internal.h"
#include "special.h"

namespace hsb {

namespace {

__device__ inline int atom_type_of(const CellArgs& c, int atom) {
  int t = 0;
  while (t + 1 < c.n_types && atom >= c.type_start[t + 1]) ++t;
  return t;
}

__device__ inline void kvec_of(const CellArgs& c, const int32_t* g, int G, double& kx, double& ky, double& kz) {
  const double n0 = g[3 * G + 0] + c.kfrac[0];
  const double n1 = g[3 * G + 1] + c.kfrac[1];
  const double n2 = g[3 * G + 2] + c.kfrac[2];
  kx = n0 * c.bvec[0] + n1 * c.bvec[3] + n2 * c.bvec[6];
  ky = n0 * c.bvec[1] + n1 * c.bvec[4] + n2 * c.bvec[7];
  kz = n0 * c.bvec[2] + n1 * c.bvec[5] + n2 * c.bvec[8];
}

// blockIdx.y == 0: K vectors and angular factors; blockIdx.y == t+1: (a_l, b_l) of type t.
__global__ void __launch_bounds__(64) k_tables(CellArgs c, const TypeConsts* __restrict__ consts, int n, int n_pad,
                                               const int32_t* __restrict__ g, double2* __restrict__ ang,
                                               double2* __restrict__ ab, double* __restrict__ kv) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= n_pad) return;
  const int part = blockIdx.y;
  const bool valid = G < n;
  double kx = 0.0, ky = 0.0, kz = 0.0;
  if (valid) kvec_of(c, g, G, kx, ky, kz);
  const double kn = sqrt(kx * kx + ky * ky + kz * kz);
  if (part == 0) {
    kv[4 * (int64_t)G + 0] = kx;
    kv[4 * (int64_t)G + 1] = ky;
    kv[4 * (int64_t)G + 2] = kz;
    kv[4 * (int64_t)G + 3] = kn;
    if (valid) {
      angular_visit(c.l_max, kx, ky, kz, c.pre, [&](int L, double re, double im) {
        ang[(int64_t)L * n_pad + G] = make_double2(re, im);
      });
    } else {
      for (int L = 0; L < c.n_l; ++L) ang[(int64_t)L * n_pad + G] = make_double2(0.0, 0.0);
    }
    return;
  }
  const int t = part - 1;
  double j[kMaxL + 2], dj[kMaxL + 1];
  if (valid) {
    sph_bessel_seq(c.l_max + 1, kn * c.r_mt[t], j);
    sph_bessel_deriv(c.l_max, j, dj);
  }
  for (int l = 0; l <= c.l_max; ++l) {
    double a = 0.0, b = 0.0;
    if (valid) {
      const double u = consts->radial[t][l][0], du = consts->radial[t][l][1];
      const double ud = consts->radial[t][l][2], dud = consts->radial[t][l][3];
      const double det = u * dud - ud * du;
      const double val = j[l], slope = kn * dj[l];
      a = (val * dud - ud * slope) / det;
      b = (u * slope - du * val) / det;
    }
    ab[((int64_t)t * (c.l_max + 1) + l) * n_pad + G] = make_double2(a, b);
  }
}

__global__ void __launch_bounds__(256) k_lambda(CellArgs c, const TypeConsts* __restrict__ consts, int K_pad,
                                                double* __restrict__ lam) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K_pad) return;
  const int rows = 2 * c.n_l;
  const int atom = k / rows, r = k % rows;
  double v = 0.0;
  if (atom < c.n_atoms) {
    if (r < c.n_l) {
      v = 1.0;
    } else {
      const int L = r - c.n_l;
      int l = 0;
      while ((l + 1) * (l + 1) <= L) ++l;
      v = consts->udot2[atom_type_of(c, atom)][l];
    }
  }
  lam[k] = v;
}

// One thread per G and a group of kAtomGroup atoms (blockIdx.y): each angular
// factor is read once and written out for every atom of the group.  Stores are
// 16 B per lane, contiguous along G.
constexpr int kAtomGroup = 8;

__global__ void __launch_bounds__(256) k_assemble(CellArgs c, int n_pad, const double2* __restrict__ ang,
                                                  const double2* __restrict__ ab, const double* __restrict__ kv,
                                                  const double* __restrict__ tau, double2* __restrict__ out,
                                                  int64_t ld, int n_store, int rows_per_atom, int64_t b_off) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  const int a0 = blockIdx.y * kAtomGroup;
  const int na = min(kAtomGroup, c.n_atoms - a0);
  if (G >= n_store) return;
  const double kx = kv[4 * (int64_t)G + 0], ky = kv[4 * (int64_t)G + 1], kz = kv[4 * (int64_t)G + 2];
  double pc[kAtomGroup], ps[kAtomGroup];
  const double2* abt[kAtomGroup];
#pragma unroll
  for (int q = 0; q < kAtomGroup; ++q) {
    const int atom = a0 + (q < na ? q : 0);
    const double arg = kx * tau[3 * atom + 0] + ky * tau[3 * atom + 1] + kz * tau[3 * atom + 2];
    sincos(arg, &ps[q], &pc[q]);
    abt[q] = ab + (int64_t)atom_type_of(c, atom) * (c.l_max + 1) * n_pad + G;
  }
  const int rows = rows_per_atom;
  int L = 0;
  for (int l = 0; l <= c.l_max; ++l) {
    double par[kAtomGroup], pai[kAtomGroup], pbr[kAtomGroup], pbi[kAtomGroup];
#pragma unroll
    for (int q = 0; q < kAtomGroup; ++q) {
      const double2 m = abt[q][(int64_t)l * n_pad];
      // phase * (a|b): complex times real
      par[q] = pc[q] * m.x; pai[q] = ps[q] * m.x;
      pbr[q] = pc[q] * m.y; pbi[q] = ps[q] * m.y;
    }
    for (int mm = 0; mm < 2 * l + 1; ++mm, ++L) {
      const double2 y = ang[(int64_t)L * n_pad + G];
#pragma unroll
      for (int q = 0; q < kAtomGroup; ++q) {
        if (q < na) {
          const int64_t rowA = (int64_t)(a0 + q) * rows + L;
          out[rowA * ld + G] = make_double2(par[q] * y.x - pai[q] * y.y, par[q] * y.y + pai[q] * y.x);
          out[(rowA + b_off) * ld + G] = make_double2(pbr[q] * y.x - pbi[q] * y.y, pbr[q] * y.y + pbi[q] * y.x);
        }
      }
    }
  }
}

// X = U B over the stacked B rows (atom, L): row r scaled by ||udot_l|| of the atom's type.
__global__ void __launch_bounds__(256) k_udot_scale(CellArgs c, const TypeConsts* __restrict__ consts, int n_pad,
                                                    const double2* __restrict__ B, double2* __restrict__ X) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= n_pad) return;
  const int rows = c.n_atoms * c.n_l;
  for (int r = blockIdx.y; r < rows; r += gridDim.y) {
    const int atom = r / c.n_l, L = r % c.n_l;
    int l = 0;
    while ((l + 1) * (l + 1) <= L) ++l;
    const double u = sqrt(consts->udot2[atom_type_of(c, atom)][l]);
    const double2 v = B[(int64_t)r * n_pad + G];
    X[(int64_t)r * n_pad + G] = make_double2(u * v.x, u * v.y);
  }
}

// Representatives of inversion pairs: tau_rep[r] = tau[rep[r]], wrow[k] = w[k / rows] for
// the k < n_rep rows stacked rows (0 on pad rows), lam[k] *= wrow[k].
__global__ void __launch_bounds__(256) k_rep_setup(const double* __restrict__ tau, const int* __restrict__ rep,
                                                   const double* __restrict__ w, int n_rep, int rows, int K_pad,
                                                   double* __restrict__ tau_rep, double* __restrict__ wrow,
                                                   double* __restrict__ lam) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_rep) {
    const int a = rep[k];
    tau_rep[3 * k + 0] = tau[3 * a + 0];
    tau_rep[3 * k + 1] = tau[3 * a + 1];
    tau_rep[3 * k + 2] = tau[3 * a + 2];
  }
  if (k < K_pad && lam) {
    const double v = k < n_rep * rows ? w[k / rows] : 0.0;
    wrow[k] = v;
    lam[k] *= v;
  }
}

__global__ void __launch_bounds__(256) k_conj(double2* __restrict__ a, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) a[i].y = -a[i].y;
}

// Caller-given coefficients [rows][ng] into the padded layout [rows][n_pad] (zeros for G >= ng).
__global__ void __launch_bounds__(256) k_pack_rows(const double2* __restrict__ src, int ng, int rows,
                                                   double2* __restrict__ dst, int n_pad) {
  const int G = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (G >= n_pad || r >= rows) return;
  dst[(int64_t)r * n_pad + G] = G < ng ? src[(int64_t)r * ng + G] : make_double2(0.0, 0.0);
}

__global__ void __launch_bounds__(256) k_zero_rows(double2* __restrict__ a, int64_t ld, int row0, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  a[(int64_t)row0 * ld + i] = make_double2(0.0, 0.0);
}

}  // namespace

hipError_t launch_tables(const CellArgs& c, const TypeConsts* consts, int n, int n_pad, const int32_t* g,
                         double2* ang, double2* ab, double* kv, hipStream_t s) {
  dim3 grid((n_pad + 63) / 64, 1 + c.n_types);
  hipLaunchKernelGGL(k_tables, grid, dim3(64), 0, s, c, consts, n, n_pad, g, ang, ab, kv);
  return hipGetLastError();
}

hipError_t launch_lambda(const CellArgs& c, const TypeConsts* consts, int K_pad, double* lam, hipStream_t s) {
  hipLaunchKernelGGL(k_lambda, dim3((K_pad + 255) / 256), dim3(256), 0, s, c, consts, K_pad, lam);
  return hipGetLastError();
}

hipError_t launch_assemble(const CellArgs& c, int n_pad, const double2* ang, const double2* ab, const double* kv,
                           const double* tau, double2* out, int64_t ld, int n_store, hipStream_t s) {
  dim3 grid((n_store + 255) / 256, (c.n_atoms + kAtomGroup - 1) / kAtomGroup);
  hipLaunchKernelGGL(k_assemble, grid, dim3(256), 0, s, c, n_pad, ang, ab, kv, tau, out, ld, n_store, 2 * c.n_l,
                     (int64_t)c.n_l);
  return hipGetLastError();
}

hipError_t launch_assemble_split(const CellArgs& c, int n_pad, const double2* ang, const double2* ab, const double* kv,
                                 const double* tau, double2* out, int64_t ld, int n_store, hipStream_t s) {
  dim3 grid((n_store + 255) / 256, (c.n_atoms + kAtomGroup - 1) / kAtomGroup);
  hipLaunchKernelGGL(k_assemble, grid, dim3(256), 0, s, c, n_pad, ang, ab, kv, tau, out, ld, n_store, c.n_l,
                     (int64_t)c.n_atoms * c.n_l);
  return hipGetLastError();
}

hipError_t launch_rep_setup(const double* tau, const int* rep, const double* w, int n_rep, int rows, int K_pad,
                            double* tau_rep, double* wrow, double* lam, hipStream_t s) {
  const int n = n_rep > K_pad ? n_rep : K_pad;
  hipLaunchKernelGGL(k_rep_setup, dim3((n + 255) / 256), dim3(256), 0, s, tau, rep, w, n_rep, rows, K_pad, tau_rep,
                     wrow, lam);
  return hipGetLastError();
}

hipError_t launch_conj(double2* a, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_conj, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, a, count);
  return hipGetLastError();
}

hipError_t launch_udot_scale(const CellArgs& c, const TypeConsts* consts, int n_pad, const double2* B, double2* X,
                             hipStream_t s) {
  const int rows = c.n_atoms * c.n_l;
  dim3 grid((n_pad + 255) / 256, rows < 1024 ? rows : 1024);
  hipLaunchKernelGGL(k_udot_scale, grid, dim3(256), 0, s, c, consts, n_pad, B, X);
  return hipGetLastError();
}

hipError_t launch_pack_rows(const double2* src, int ng, int rows, double2* dst, int n_pad, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_rows, dim3(n_pad / 256 + (n_pad % 256 ? 1 : 0), rows), dim3(256), 0, s, src, ng, rows, dst,
                     n_pad);
  return hipGetLastError();
}

hipError_t launch_zero_rows(double2* a, int64_t ld, int row0, int row1, hipStream_t s) {
  if (row1 <= row0) return hipSuccess;
  const int64_t count = (int64_t)(row1 - row0) * ld;
  hipLaunchKernelGGL(k_zero_rows, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, a, ld, row0, count);
  return hipGetLastError();
}

}  // namespace hsb
