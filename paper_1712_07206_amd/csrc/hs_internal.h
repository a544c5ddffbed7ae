// Internal declarations shared by the host library and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>

#include "hsbuild.h"

namespace hsb {

constexpr int kTileN = 128;  // basis sizes are padded to a multiple of this
constexpr int kTileK = 16;   // the stacked contraction index is padded to a multiple of this

// Rows of the stacked operands: K plus at least kTileK - 1 zero rows, so the per-atom T
// products, which read an atom's rows in kTileK-row chunks, stay inside the array for
// the last atom.
inline int stacked_pad(int K) { return (K + 2 * kTileK - 2) / kTileK * kTileK; }
// Shape of the zero-padded transposed T of one type (2N_L = M): [tprod_kc(M)][tprod_mp(M)].
inline int tprod_kc(int M) { return (M + 15) / 16 * 16; }
inline int tprod_mp(int M) { return (M + 127) / 128 * 128; }

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Cell description passed by value to the coefficient kernels.
struct CellArgs {
  double bvec[9];   // reciprocal basis rows b_j (a_i . b_j = 2 pi delta_ij)
  double kfrac[3];  // k in the reciprocal basis
  double pre;       // 4 pi / sqrt(Omega)
  int n_types, n_atoms, l_max, n_l;
  int type_start[HSB_MAX_TYPES + 1];  // atoms of type t: [type_start[t], type_start[t+1])
  double r_mt[HSB_MAX_TYPES];
};

// Device-side per-type constants, copied into the workspace by each call.
struct TypeConsts {
  double radial[HSB_MAX_TYPES][HSB_MAX_LMAX + 1][4];  // u, u', udot, udot' at R_MT
  double udot2[HSB_MAX_TYPES][HSB_MAX_LMAX + 1];      // ||udot_l||^2
};

// Placement of one k-point's arrays inside the workspace (byte offsets).
//   W   : stacked coefficients, complex [K_pad][n_pad]; row k = (atom, A|B, L)
//         = atom*2N_L + (0 for A, N_L for B) + L; columns G (>= n are zero)
//   Y   : T_t W per atom, same shape (rows >= K are zero)
//   ang : pre * i^l conj(Y_lm(K_hat_G)), complex [N_L][n_pad]
//   ab  : (a_l, b_l) per type, double2 [n_types][l_max+1][n_pad]
//   kv  : (Kx, Ky, Kz, |K|) per G, double4-like [n_pad][4]
//   lam : S weight of row k (1 for A rows, ||udot_l||^2 for B rows, 0 for pad)
struct Layout {
  int n = 0, n_pad = 0, K = 0, K_pad = 0;
  size_t W = 0, Y = 0, ang = 0, ab = 0, kv = 0, lam = 0, consts = 0, end = 0;
  size_t WL = 0;  // lam W (the FP64 contraction's S operand), forward in FP64 only
  int ns = 1;              // FP64 forward: segments of the stacked index (split contraction when > 1)
  int nsh = 0;             // FP64 forward: workgroups of the stream-K contraction (0: not used)
  size_t skH = 0, skS = 0;  // partial H and S: per segment (ns > 1), or the stream-K slots (nsh > 0)
  size_t PH = 0, PS = 0, partT = 0, partTau = 0;  // backward only
  size_t WT = 0, gHp = 0, gSp = 0;                // backward: operands of the 3M products
  size_t TT = 0;                                  // T^T per type, zero-padded (T products)
  int Kt = 0;                                     // backward: K_pad rounded up to 128
  int K_pad2 = 0;                                  // split only: stacked rows padded to 32
  size_t mx = 0, scale = 0, slL = 0, slS = 0, slY = 0;  // split only (slL, slS, slY: residue planes in the CRT form)
  int K64 = 0, n_res = 0;                              // residue form: rows padded to 64, columns to 256
  size_t crPart = 0, crRes = 0, crResH = 0;            // residue form: partial column norms, residues of S, H
  // factored only: rows [R_f] of X (E and W0 blocks), XL = lam X, Yx (Y0 on W0 rows, 0 on E rows)
  int R_f = 0;
  size_t X = 0, XL = 0, Yx = 0, lamx = 0, kind = 0, tau0 = 0;
  // BLAS baseline only: A and B stacks, X scratch, rocBLAS's device memory
  size_t hA = 0, hB = 0, hX = 0, blas = 0, blas_bytes = 0;
  // real-symmetric only: representative indices and weights, their positions, row weights
  size_t rep = 0, repw = 0, tau_rep = 0, wrow = 0;
  // eigensolve only: rocSOLVER's off-diagonal scratch
  size_t eigE = 0;
};

// Per-k-point entry of the batched contraction's tile list (device copy in the workspace).
struct BatchMeta {
  int64_t w_off, wl_off, y_off;  // W_k, lam W_k and Y_k, in complex elements from the workspace base
  int64_t out_off;       // H_k, S_k, in complex elements from the output bases (ld = n)
  int n, n_pad, nbr, tile_start;
};

// ---- kernel launchers (each returns hipGetLastError() after enqueue) ----

// ang, ab, kv (all padded columns written) from the G list.
hipError_t launch_tables(const CellArgs& c, const TypeConsts* consts, int n, int n_pad, const int32_t* g,
                         double2* ang, double2* ab, double* kv, hipStream_t s);
// lam[k] for k in [0, K_pad).
hipError_t launch_lambda(const CellArgs& c, const TypeConsts* consts, int K_pad, double* lam, hipStream_t s);
// out[(atom*2N_L + (A|B)*N_L + L) * ld + G] for G < n_store.
hipError_t launch_assemble(const CellArgs& c, int n_pad, const double2* ang, const double2* ab, const double* kv,
                           const double* tau, double2* out, int64_t ld, int n_store, hipStream_t s);
// The same with A and B in separate stacks: A rows atom*N_L + L, B rows N_atoms*N_L + atom*N_L + L.
hipError_t launch_assemble_split(const CellArgs& c, int n_pad, const double2* ang, const double2* ab, const double* kv,
                                 const double* tau, double2* out, int64_t ld, int n_store, hipStream_t s);
// Inversion pairs: tau_rep[r] = tau[rep[r]] (r < n_rep); with lam non-null, wrow[k] = w[k / rows]
// over the stacked rows (0 for k >= n_rep rows) and lam[k] *= wrow[k], k < K_pad.
hipError_t launch_rep_setup(const double* tau, const int* rep, const double* w, int n_rep, int rows, int K_pad,
                            double* tau_rep, double* wrow, double* lam, hipStream_t s);
// X = U B over the stacked B rows (atom, L), U = diag(||udot_l||) of the atom's type.
hipError_t launch_udot_scale(const CellArgs& c, const TypeConsts* consts, int n_pad, const double2* B, double2* X,
                             hipStream_t s);
// dst[r][G] = src[r][G] for G < ng, 0 up to n_pad (rows r < rows; rows <= 65535).
hipError_t launch_pack_rows(const double2* src, int ng, int rows, double2* dst, int n_pad, hipStream_t s);
// rows [row0, row1) of a [*][ld] complex array set to zero.
hipError_t launch_zero_rows(double2* a, int64_t ld, int row0, int row1, hipStream_t s);
// Y_atom = T_type(atom) W_atom for every atom (rows of W/Y per atom: 2N_L).
hipError_t launch_tprod(const CellArgs& c, const double2* TT, const double2* W, double2* Y, int n_pad,
                        hipStream_t s);
// TT[t] = T[t]^T zero-padded to [tprod_kc(M)][tprod_mp(M)] for each of n_types types (M = 2 N_L).
hipError_t launch_tpad(const double2* T, int n_types, int M, double2* TT, hipStream_t s);
// Y_a = T_t(a) W_a for every atom of c from TT, in the 3M form (k_hs.hip).
hipError_t launch_tprod3m(const CellArgs& c, const double2* TT, const double2* W, double2* Y, int n_pad,
                          hipStream_t s);
// Upper triangles of H = W^H Y and S = W^H WL over K_pad rows (WL = diag(lam) W, prepared).
// gr: tile order (0 row-major, > 0 super-rows taken in groups of gr).
// waves: 4 (64 x 32 per wave) or 8 (32 x 32 per wave).
// waves 8: three real MFMAs per complex multiply-add (3M form, operands WL and Y); waves 4: the plain
// four-MFMA form (lam applied to W while staging).
hipError_t launch_hs_fp64(const double2* W, const double2* WL, const double2* Y, const double* lam, int K_pad, int n,
                          int n_pad, int gr, int waves, double2* H, double2* S, int64_t ldh, hipStream_t s);

// Stream-K form of the 8-wave FP64 contraction, for an upper triangle of fewer than 4 tiles per
// compute unit: the number of workgroups (shares, each of at least 256 stacked rows, at most one
// per compute unit) when a time model puts it ahead of one pass, else 0.
int hs_stream_shares(int n_pad, int K_pad, int num_cus);
// Elements of each of its partial-tile buffers Hp, Sp: two 128 x 64 slots per share.
size_t hs_stream_slot_elems(int nsh);
// The (tile, 16-row chunk) units in nsh equal contiguous shares: whole tiles into H, S (ldh), the
// pieces of tiles shared between workgroups into Hp, Sp; launch_stream_fixup adds each shared
// tile's pieces in chunk order into H, S (upper triangle, row <= col < n).  The tiles are taken in
// one fixed order, so the results do not depend on the tile-order option.
hipError_t launch_hs_fp64_stream(const double2* W, const double2* WL, const double2* Y, int K_pad, int nsh, int n,
                                 int n_pad, double2* H, double2* S, int64_t ldh, double2* Hp, double2* Sp,
                                 hipStream_t s);
hipError_t launch_stream_fixup(int K_pad, int nsh, int n, int n_pad, const double2* Hp, const double2* Sp,
                               double2* H, double2* S, int64_t ldh, hipStream_t s);
// Rows per segment (a multiple of the 16-row chunk; the last segment takes the rest).
int hs_split_rows(int K_pad, int ns);
// The 8-wave (3M) contraction in ns segments of the stacked index: partial tiles into Hp, Sp
// ([ns][n_pad][n_pad] each); launch_sk_reduce then sets H, S = the segments added in order
// (upper triangle, row <= col < n).
hipError_t launch_hs_fp64_sk(const double2* W, const double2* WL, const double2* Y, int K_pad, int ns, int n,
                             int n_pad, int gr, double2* Hp, double2* Sp, hipStream_t s);
hipError_t launch_sk_reduce(const double2* Hp, const double2* Sp, int ns, int n, int n_pad, double2* H, double2* S,
                            int64_t ldh, hipStream_t s);

// The same contraction keeping only the real parts, Re(W^H Y) and Re(W^H lam W), as doubles.
hipError_t launch_hs_fp64_real(const double2* W, const double2* WL, const double2* Y, const double* lam, int K_pad,
                               int n, int n_pad, int gr, int waves, double* H, double* S, int64_t ldh, hipStream_t s);

// Number of 128 x 64 tiles the contraction covers for a padded basis size.
int hs_tiles(int n_pad);
// Persistent contraction over the tiles of every k-point in meta (grid: a multiple of 8).
hipError_t launch_hs_fp64_batch(const double2* ws, const double* lam, int K_pad, const BatchMeta* meta, int n_k,
                                int total, int grid, int gr, int waves, double2* H, double2* S, hipStream_t s);

// ---- matrix-core rate probe (kind 0: FP64 16x16x4, 1: int8 32x32x32) ----
constexpr int kProbeUnroll = 16;  // iterations per loop pass: the probe's iters must be a multiple
double probe_ops_per_mfma(int kind);
hipError_t launch_mfma_probe(int kind, int blocks, int iters, void* out, hipStream_t s);

// ---- split precision ----
// Column scales 2^e (max_k |Re|, |Im| < 2^e) of W, lam W and Y: scale[0..3 n_pad); mx: 3 n_pad scratch.
hipError_t launch_split_scales(const double2* W, const double2* Y, const double* lam, int K, int n_pad,
                               unsigned long long* mx, double* scale, hipStream_t s);
// S 8-bit slices (BF16 or FP16 values) of X (times lam if use_lam) in the blocked layout, QK = K_pad2 / 8.
hipError_t launch_split_slices(int precision, int S, const double2* X, const double* lam, int use_lam, int K,
                               int n_pad, int QK, const double* scale, void* out, hipStream_t s);
// Upper triangle of C = conj(L)^T R from the slices (C: [n][n]).
// int8 slices only: C = Re(conj(L)^T R) into a real [n][n] array, upper triangle
hipError_t launch_hs_split8_real(int S, const void* L, const void* R, const double* scL, const double* scR, int QK,
                                 int n, int n_pad, int gr, double* C, hipStream_t s);
hipError_t launch_hs_split(int precision, int S, const void* L, const void* R, const double* scL, const double* scR,
                           int QK, int n, int n_pad, int gr, double2* C, hipStream_t s);

// ---- split precision by residues (Chinese remainder) ----
// At most 13 moduli: M < 2^97, so the scaled integer operands stay below 2^48 (the residue
// kernel's exact reduction needs that).
constexpr int kCrtMinModuli = 8, kCrtMaxModuli = 13;
constexpr int kCrtRows = 64;  // stacked rows per stage of the residue contraction (K padded to it)
// Moduli and recombination constants, passed to the kernels by value.
struct CrtConsts {
  int n_mod;
  int m[kCrtMaxModuli];      // coprime moduli, each a power of a prime p = 1 (mod 4), below 256
  int j[kCrtMaxModuli];      // j^2 = -1 (mod m)
  int inv2[kCrtMaxModuli];   // 2^{-1} (mod m)
  int inv2j[kCrtMaxModuli];  // (2 j)^{-1} (mod m)
  double h[kCrtMaxModuli];   // y_i / m_i = h_i + l_i, y_i = (M / m_i)^{-1} (mod m_i), h_i on a 2^-42 grid
  double l[kCrtMaxModuli];
  // the same split of (2^{-1} y_i mod m_i) / m_i and ((2 j)^{-1} y_i mod m_i) / m_i on a 2^-41 grid:
  // the weights of P + Q and P - Q, whose residues need no reduction
  double h_re[kCrtMaxModuli], l_re[kCrtMaxModuli];
  double h_im[kCrtMaxModuli], l_im[kCrtMaxModuli];
  double M;                  // product of the moduli (rounded)
  double bound;              // largest 2-norm of a scaled integer column: bound^2 < M/2 (1 - 2^-10)
};
// Host: the n_mod largest such moduli and their constants; false if n_mod is out of range.
bool crt_make_consts(int n_mod, CrtConsts* cc);
// Residue columns: the basis padded to whole 256-row tiles.
inline int crt_cols(int n) { return (int)round_up(n, 256); }
int crt_norm_blocks(int K);
int crt_tiles(int n_res);
// Column scales (powers of two) of W, lam W and Y: scale[0..3 n_res); part: 3 crt_norm_blocks(K) n_res doubles.
hipError_t launch_crt_scales(const double2* W, const double2* Y, const double* lam, int K, int n_pad, int n_res,
                             const CrtConsts& cc, double* part, double* scale, hipStream_t s);
// Element kind of the residues: signed bytes on the int8 MFMA (HSB_SPLIT_CRT), bfloat16
// (HSB_SPLIT_CRT_BF16) or half (HSB_SPLIT_CRT_FP16) integers on the 16-bit MFMAs.
inline int crt_kind(int precision) {
  return precision == HSB_SPLIT_CRT_BF16 ? 1 : precision == HSB_SPLIT_CRT_FP16 ? 2 : 0;
}
inline bool is_crt(int precision) {
  return precision == HSB_SPLIT_CRT || precision == HSB_SPLIT_CRT_BF16 || precision == HSB_SPLIT_CRT_FP16;
}
// Stacked rows per 16-byte residue unit: 16 bytes, or 8 16-bit elements.
inline int crt_unit_rows(int ek) { return ek == 0 ? 16 : 8; }
// Residue planes of X (times lam if use_lam): per modulus [QK / 4][n_res / 64][2][4][64] 16-byte units
// (chunk-major), QK = K64 / crt_unit_rows(ek).
hipError_t launch_crt_residues(const CrtConsts& cc, int ek, const double2* X, const double* lam, int use_lam, int K,
                               int n_pad, int n_res, int QK, const double* scale, void* out, hipStream_t s);
// Residues of the upper triangle of conj(L)^T R per modulus: res [n_mod][2][n_res][n_res] signed
// bytes, P then Q (the images of the product under the two factors of Z[i]/m); the real form
// [n_mod][n_res][n_res], its one product.  256 x 256 blocks; waves: 8 (waves of 64 x 128) or
// 4 (128 x 128).
hipError_t launch_hs_crt(const CrtConsts& cc, int ek, bool real, const void* L, const void* R, int QK, int n,
                         int n_res, int gr, int waves, void* res, hipStream_t s);
// C[row][col] (row <= col < n, ld n) from the residues (Re, Im from P, Q per modulus), scaled by
// 1 / (scL[row] scR[col]); complex or real.
hipError_t launch_crt_combine(const CrtConsts& cc, bool real, const void* res, int n_res, const double* scL,
                              const double* scR, int n, void* C, hipStream_t s);

// ---- type-factored form ----
// Number of 64 x 64 tiles of the factored contraction.
int fact_tiles(int n_pad);
// E[a][G] = e^{i K_G . tau_a}, rows a < n_atoms of a [*][n_pad] array.
hipError_t launch_phases(int n_atoms, int n_pad, const double* kv, const double* tau, double2* E, hipStream_t s);
// Row blocks of the factored layout: per type with atoms, round16(N_t) E rows then
// round16(2 N_L) W0 rows.  lamx[r] and the kind of every 16-row chunk.
hipError_t launch_fact_rows(const CellArgs& c, const TypeConsts* consts, int rows, double* lamx, int* kind,
                            hipStream_t s);
// XL[r][G] = lam[r] X[r][G] for r < rows.
hipError_t launch_scale_rows(const double2* X, const double* lam, int rows, int n_pad, double2* XL, hipStream_t s);
// Upper triangles of H = sum_t P_t * (W0_t^H Y0_t), S = sum_t P_t * (W0_t^H Lam_t W0_t), P_t = E_t^H E_t,
// from the per-type row blocks of X, XL = lam X and Yx (nch chunks of 16 rows, kinds in kind[]).
hipError_t launch_hs_fact(const double2* X, const double2* XL, const double2* Yx, const int* kind, int nch, int n,
                          int n_pad, int gr, double2* H, double2* S, int64_t ldh, hipStream_t s);

// ---- the paper's algorithm on rocBLAS (baseline) ----
int hsdla_blas_create(int device, void** handle, std::string& err);
void hsdla_blas_destroy(void* handle);
int hsdla_blas_workspace(void* handle, int algorithm, const CellArgs& c, int ng, int n_pad, size_t* bytes,
                         std::string& err);
int hsdla_blas_bind(void* handle, void* ws, size_t bytes, hipStream_t s, std::string& err);
int hsdla_blas_enqueue(void* handle, int algorithm, const CellArgs& c, const TypeConsts* consts, int ng, int n_pad,
                       const double2* T, const double2* A, const double2* B, double2* X, double2* H, double2* S,
                       hipStream_t s, bool query, std::string& err);

int eig_enqueue(void* handle, int n, double2* H, double2* S, double* w, double* E, int* info, bool vectors,
                std::string& err);
int eig_workspace(void* handle, int n, bool vectors, size_t* bytes, std::string& err);
// a[i] = conj(a[i]) for i < count.
hipError_t launch_conj(double2* a, int64_t count, hipStream_t s);

// ---- adjoint ----
int gradtau_blocks(int n);
// P_H = W gH and P_S = W gS ([K_pad][n_pad]) in the 3M form from W^T ([n_pad][Kt], Kt a multiple
// of 128, zeros past K_pad) and gS, gH zero-padded to [n_pad][n_pad].
hipError_t launch_pgemm3m(const double2* WT, const double2* gSp, const double2* gHp, int Kt, int K_pad, int n_pad,
                          double2* PH, double2* PS, hipStream_t s);
// WT[G][k] = W[k][G] (k < K_pad), 0 for K_pad <= k < Kt.
hipError_t launch_transpose(const double2* W, int K_pad, int n_pad, int Kt, double2* WT, hipStream_t s);
// gp = g ([n][n]) zero-padded to [n_pad][n_pad].
hipError_t launch_pad_square(const double2* g, int n, int n_pad, double2* gp, hipStream_t s);
// gT[t] = sum over atoms of type t of P_H,a W_a^H (part: [n_atoms][2N_L][2N_L] scratch).
hipError_t launch_gradT(const CellArgs& c, const double2* PH, const double2* W, int n_pad, double2* part,
                        double2* gT, hipStream_t s);
// gtau[a] = -2 sum_G K_G Im c_a(G) (part: [n_atoms][gradtau_blocks(n)][3] scratch).
hipError_t launch_gradtau(const CellArgs& c, const double2* PH, const double2* PS, const double2* Y,
                          const double2* W, const double* lam, const double* kv, int n, int n_pad, double* part,
                          double* gtau, hipStream_t s);

}  // namespace hsb
