/*
 * hsbuild: muffin-tin Hamiltonian and overlap matrices of the FLAPW method on
 * one AMD Instinct MI355X (gfx950).
 *
 * For one k-point with plane-wave basis {G : |k+G| <= K_max} (Sec. 2.1 of
 * Davidovic et al., "Accelerating the computation of FLAPW methods on
 * heterogeneous architectures"), the library builds the complex Hermitian
 * N_G x N_G matrices
 *
 *   S = sum_a A_a^H A_a + B_a^H diag(||udot_l||^2) B_a            (Eq. 4 / Eq. 7)
 *   H = sum_a [A_a; B_a]^H T_t(a) [A_a; B_a]                       (Eq. 5 / Eq. 6)
 *
 * where a runs over atoms, t(a) is the atom's type, A_a, B_a in C^{N_L x N_G}
 * are the matching coefficients of Eq. 2 and T_t = [[T^AA, T^AB], [T^BA, T^BB]]
 * (T^BA = (T^AB)^H, Sec. 3) is the type's 2N_L x 2N_L Hermitian block.
 *
 * Matching coefficients (Eq. 2 with continuity of value and slope at R_MT,
 * Sec. 2.1; the paper leaves the formula to the standard LAPW matching):
 *   K = k + G, x = |K| R_t, W_l = u udot' - udot u'
 *   a_l = (j_l(x) udot' - |K| j_l'(x) udot) / W_l,  b_l = (|K| j_l'(x) u - j_l(x) u') / W_l
 *   A^{a,G}_{lm} = (4 pi / sqrt(Omega)) e^{i K.tau_a} i^l conj(Y_lm(K_hat)) a_l,  B likewise with b_l
 * Y_lm: complex orthonormal spherical harmonics with the Condon-Shortley
 * phase; compound index L = l^2 + l + m, m = -l..l.  K_hat = z when |K| < 1e-12.
 *
 * Conventions for every entry point:
 *   - complex values are complex128, interleaved (re, im) doubles;
 *   - matrices are row-major; H and S are indexed [G'][G] in the caller's G
 *     order, leading dimension N_G; only the upper triangle (column >= row,
 *     diagonal included) is written, the strict lower triangle is untouched
 *     (exceptions: hsbuild_forward_real writes doubles, and algorithm 1 of
 *     hsbuild_forward_hsdla writes both triangles of H);
 *   - all arguments are validated on the host before anything is enqueued; on
 *     an error nothing is launched and the outputs are untouched;
 *   - calls are asynchronous and stream-ordered on `stream` (a hipStream_t,
 *     NULL = the default stream); device faults surface at the caller's
 *     synchronisation;
 *   - the caller owns every device buffer, the workspace included; the
 *     library's kernels allocate no device memory (the rocBLAS/rocSOLVER
 *     paths bind the vendor library to a region of the caller's workspace;
 *     the rocBLAS handle itself is created by rocBLAS the first time a handle
 *     sizes or runs hsbuild_forward_hsdla or hsbuild_eigensolve);
 *   - a handle is not thread-safe: use one handle per stream.
 */
#ifndef HSBUILD_H
#define HSBUILD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hsbuild_s* hsbuild_t;

/* Status codes. */
enum {
  HSB_OK = 0,
  HSB_ERR_ARG = -1,         /* null pointer, out-of-range scalar */
  HSB_ERR_SHAPE = -2,       /* inconsistent sizes (e.g. ng > max_ng) */
  HSB_ERR_WORKSPACE = -3,   /* workspace smaller than hsbuild_workspace_bytes() */
  HSB_ERR_DEVICE = -4,      /* no usable gfx950 device, or a launch error */
  HSB_ERR_UNSUPPORTED = -5, /* valid request the library does not implement */
  HSB_ERR_NUMERIC = -6      /* singular radial Wronskian at create */
};

/* Contraction precision.  The slice forms cut every operand column, scaled by a
 * power of two, into n_slices integer slices and run the slice products on the
 * matrix cores: 8-bit slices as BF16 or FP16 values with FP32 sums, or 7-bit
 * slices as signed bytes with exact int32 sums (HSB_SPLIT_INT8).  The residue
 * form (HSB_SPLIT_CRT) rounds every column, scaled by a power of two, to
 * Gaussian integers, multiplies their residues modulo n_slices coprime moduli
 * below 256 on the int8 matrix cores (exact int32 sums, two products per
 * modulus for a complex product) and recovers the integer products by the
 * Chinese remainder theorem in FP64.  HSB_SPLIT_CRT_BF16 and
 * HSB_SPLIT_CRT_FP16 are the same residue form with the residues as bfloat16
 * or half integers on the 16-bit matrix cores (FP32 sums, exact for integers
 * below 2^24: reduced modulo each modulus every 1024 stacked rows); the three
 * give bitwise the same H and S. */
enum { HSB_FP64 = 0, HSB_SPLIT_FP16 = 1, HSB_SPLIT_BF16 = 2, HSB_SPLIT_INT8 = 3, HSB_SPLIT_CRT = 4,
       HSB_SPLIT_CRT_BF16 = 5, HSB_SPLIT_CRT_FP16 = 6 };

/* Workspace modes for hsbuild_workspace_bytes. */
enum { HSB_MODE_FORWARD = 0, HSB_MODE_BACKWARD = 1, HSB_MODE_BATCH = 2, HSB_MODE_COEFFICIENTS = 3, HSB_MODE_FACTORED = 4,
       HSB_MODE_HSDLA = 5, HSB_MODE_REAL = 6, HSB_MODE_EIGEN = 7 };

#define HSB_MAX_TYPES 16
#define HSB_MAX_LMAX 12

/* Static description of the cell; all pointers are host memory and are
 * copied by hsbuild_create (the caller may free them afterwards). */
typedef struct {
  int32_t n_types;            /* 1..HSB_MAX_TYPES */
  int32_t n_atoms;            /* >= 1 */
  int32_t l_max;              /* 0..HSB_MAX_LMAX; N_L = (l_max+1)^2 */
  int32_t max_ng;             /* largest basis size any call will pass */
  double lattice[9];          /* rows a1, a2, a3 (bohr); Omega = |det| */
  const int32_t* atom_type;   /* [n_atoms], non-decreasing (atoms grouped by type) */
  const double* r_mt;         /* [n_types] muffin-tin radii (bohr), > 0 */
  const double* radial;       /* [n_types][l_max+1][4]: u, u', udot, udot' at R_MT */
  const double* udot_norm2;   /* [n_types][l_max+1]: ||udot_l||^2 >= 0 */
  int32_t precision;          /* HSB_FP64, HSB_SPLIT_FP16, HSB_SPLIT_BF16, HSB_SPLIT_INT8,
                                 HSB_SPLIT_CRT, HSB_SPLIT_CRT_BF16 or HSB_SPLIT_CRT_FP16 */
  int32_t n_slices;           /* split path only: slices per operand, 3..6 (8 bits each
                                 for BF16/FP16, 7 for INT8); for the residue forms
                                 (HSB_SPLIT_CRT*) the number of moduli, 8..13 (each adds
                                 about 3.7 bits per operand column; 11 keeps the error
                                 near 1e-11) */
} hsb_config;

/* Create a handle.  Returns HSB_ERR_NUMERIC if some radial Wronskian
 * |u udot' - udot u'| < 1e-12 (|u udot'| + |udot u'|), HSB_ERR_DEVICE if the
 * current device is not gfx950.  *out is set only on success. */
int hsbuild_create(const hsb_config* cfg, hsbuild_t* out);

/* Destroy a handle (NULL is ignored).  Waits only for a batch graph this
 * handle launched; other work the caller enqueued is not synchronised. */
void hsbuild_destroy(hsbuild_t h);

/* Bytes of device workspace a call needs.  mode: HSB_MODE_*; ng: host array
 * of n_k basis sizes (n_k = 1 except for HSB_MODE_BATCH).  Returns 0 on an
 * invalid request (see hsbuild_last_error). */
size_t hsbuild_workspace_bytes(hsbuild_t h, int32_t mode, int32_t n_k, const int32_t* ng);

/* Matching coefficients only (Eq. 2): coef (device, complex128
 * [n_atoms][2][N_L][ng]) receives A (index 0) and B (index 1) of every atom.
 * k_frac: host double[3], k in the reciprocal basis; g: device int32
 * [ng][3] integer reciprocal vectors; tau: device double [n_atoms][3]
 * cartesian positions (bohr). */
int hsbuild_coefficients(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g,
                         const double* tau, void* coef, void* ws, size_t ws_bytes, void* stream);

/* H and S of one k-point (Eqs. 4-7).  T: device complex128
 * [n_types][2N_L][2N_L], Hermitian, rows/columns ordered (A|B, L).
 * H, S: device complex128 [ng][ng]; upper triangle written.
 * The handle's precision selects the FP64 MFMA contraction or the
 * split-precision (Ozaki slice) contraction. */
int hsbuild_forward(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                    const void* T, void* H, void* S, void* ws, size_t ws_bytes, void* stream);

/* H and S of one k-point exactly as hsbuild_forward (same arguments, results,
 * precision handling and errors), for callers that cannot allocate device
 * memory: code under hipGraph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  There is no workspace argument: the call runs in a device
 * array the library holds, HSB_STATIC_SCRATCH_BYTES long, one copy per GPU,
 * kept from the library's first use on that GPU until the process ends.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library call).
 * A problem whose hsbuild_workspace_bytes(h, HSB_MODE_FORWARD, 1, &ng) exceeds
 * HSB_STATIC_SCRATCH_BYTES gets HSB_ERR_WORKSPACE before anything is enqueued
 * (use hsbuild_forward with a caller workspace for it).  Every call on one GPU
 * uses that GPU's one array, whose contents stay from the last call (each call
 * overwrites every byte it reads first): calls that may overlap on one GPU --
 * on different streams, from different handles or threads without ordering --
 * race and give undefined results. */
#define HSB_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
int hsbuild_forward_static(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                           const void* T, void* H, void* S, void* stream);

/* H and S of one k-point by the type-factored ("compressed") contraction,
 * the compression of A and B that Sec. 7 proposes: each atom's coefficients
 * are its type's coefficients at the origin times the structure phase
 * e^{i K_G . tau_a}, so (Eqs. 4-5)
 *   H = sum_t P_t .* (W0_t^H T_t W0_t),  S = sum_t P_t .* (W0_t^H Lam_t W0_t),
 *   P_t[G'][G] = sum over the atoms a of type t of e^{-i K_G' . tau_a} e^{i K_G . tau_a}
 * (.* entrywise), with contraction width sum_t (N_t + 4 N_L) per entry
 * instead of 4 N_atoms N_L.  Same arguments and results as hsbuild_forward
 * (equal up to FP64 rounding); always FP64, whatever the handle's precision.
 * Workspace: hsbuild_workspace_bytes(h, HSB_MODE_FACTORED, 1, &ng). */
int hsbuild_forward_factored(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                             const void* T, void* H, void* S, void* ws, size_t ws_bytes, void* stream);

/* H and S of an inversion-symmetric cell as real symmetric matrices (the
 * real case that Sec. 2.1 allows besides the complex Hermitian one).
 * partner: host int32 [n_atoms], partner[a] = the atom at -tau_a (a itself for
 * an atom at the origin); it must be an involution within each type.  The
 * caller guarantees the symmetry: tau_partner[a] = -tau_a, and each T_t
 * invariant under time reversal, T[(X,l,m),(X',l',m')] = (-1)^(m+m')
 * conj(T[(X,l,-m),(X',l',-m')]), with no entries of odd l + l'.  Then each
 * pair contributes twice the real part of one member's term, so only one atom
 * of each pair is built and the contraction keeps only real parts: about a
 * quarter of the work of hsbuild_forward.  H, S: device double [ng][ng],
 * upper triangle written; equal to the real parts of hsbuild_forward's
 * outputs up to FP64 rounding (undefined if the symmetry does not hold).
 * Other arguments as hsbuild_forward.  A handle created with HSB_FP64 runs
 * the FP64 contraction; one created with HSB_SPLIT_INT8 or a residue form
 * (HSB_SPLIT_CRT*) runs that split contraction (the real parts of the split
 * products, to the split path's error); HSB_SPLIT_BF16 and HSB_SPLIT_FP16 handles get
 * HSB_ERR_UNSUPPORTED before anything is enqueued.
 * Workspace: hsbuild_workspace_bytes(h, HSB_MODE_REAL, 1, &ng). */
int hsbuild_forward_real(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                         const int32_t* partner, const void* T, double* H, double* S, void* ws, size_t ws_bytes,
                         void* stream);

/* The paper's own algorithm on the vendor BLAS (rocBLAS), a baseline for the
 * fused kernels: A and B stacks built on the GPU as for hsbuild_forward, then
 * the BLAS-3 sequence of Alg. 3 (algorithm = 3: zherk, zherk on U B, per-atom
 * zgemm + zhemm, zher2k, per-atom zhemm, zherkx) or of Alg. 1 (algorithm = 1)
 * with H_AA by a per-atom zhemm and a general zgemm, the branch Alg. 1 takes
 * when the Cholesky factorisation of T_AA fails (as it does for T_AA with
 * negative diagonal entries).  Same H and S as hsbuild_forward up to FP64
 * rounding; algorithm 3 writes the upper triangles only, algorithm 1 writes
 * both triangles of H (its strict lower triangle is not meaningful).
 * Workspace: hsbuild_workspace_bytes(h, HSB_MODE_HSDLA, 1, &ng), which
 * includes the device memory rocBLAS asks for (the library binds it to the
 * caller's workspace). */
int hsbuild_forward_hsdla(hsbuild_t h, int32_t algorithm, const double k_frac[3], int32_t ng, const int32_t* g,
                          const double* tau, const void* T, void* H, void* S, void* ws, size_t ws_bytes,
                          void* stream);

/* The generalized eigenproblem H c = lambda S c that H and S are built for
 * (Sec. 2.1), on the vendor library (rocSOLVER zhegvd).  H, S: device
 * complex128 [ng][ng] holding the upper triangles hsbuild_forward writes; both
 * are overwritten: with vectors = 1, row j of H receives the eigenvector c_j
 * (normalised to c_j^H S c_j = 1), and S the Cholesky factor.  w: device double
 * [ng], the eigenvalues in ascending order.  info: device int32 [1], rocSOLVER's
 * status (0 = success; > ng: S is not positive definite; 1..ng: no
 * convergence) -- read it after synchronising.  S must be positive definite:
 * the muffin-tin S alone has rank <= 2 N_atoms N_L, so ng must stay below that
 * (the interstitial part that makes S definite in general is not built here).
 * Workspace: hsbuild_workspace_bytes(h, HSB_MODE_EIGEN, 1, &ng), which includes
 * the device memory rocSOLVER asks for. */
int hsbuild_eigensolve(hsbuild_t h, int32_t ng, void* H, void* S, double* w, int32_t vectors, int32_t* info, void* ws,
                       size_t ws_bytes, void* stream);

/* H and S from caller-given matching coefficients, the input the paper's
 * HSDLA algorithm starts from (Alg. 1, Alg. 3): coef is device complex128
 * [n_atoms][2][N_L][ng] (index 0: A, 1: B, as hsbuild_coefficients writes
 * it); T, H, S, workspace (HSB_MODE_FORWARD size) and precision as for
 * hsbuild_forward. */
int hsbuild_forward_coefficients(hsbuild_t h, int32_t ng, const void* coef, const void* T, void* H, void* S,
                                 void* ws, size_t ws_bytes, void* stream);

/* Adjoint of hsbuild_forward for a real loss L(H, S).  gH, gS: device
 * complex128 [ng][ng], the full Hermitian gradients dL/dRe H + i dL/dIm H
 * (likewise S).  Outputs: gT device complex128 [n_types][2N_L][2N_L] =
 * dL/dRe T + i dL/dIm T with T's entries taken as free; gtau device double
 * [n_atoms][3] = dL/dtau (cartesian).  Both outputs are overwritten.
 * The coefficients are recomputed, nothing is kept from the forward. */
int hsbuild_backward(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                     const void* T, const void* gH, const void* gS, void* gT, double* gtau, void* ws,
                     size_t ws_bytes, void* stream);

/* H and S of n_k k-points sharing tau and T: Sec. 2.1 sets up one basis, and
 * one pair H(k), S(k), per k-point of the Brillouin-zone sampling, each with
 * its own basis size N_G(k).  k_frac: host double[n_k][3]; ng: host
 * int32[n_k]; g: device int32, the n_k G lists concatenated in k order;
 * out_off: host int64[n_k], element offsets of each k's ng x ng block in H and
 * S (blocks must not overlap: HSB_ERR_SHAPE).  Each block holds exactly what
 * hsbuild_forward writes for that k (bitwise, with the same options and
 * HSB_OPT_SPLIT_K = 0; to FP64 rounding where the forward splits), upper
 * triangle only.  FP64 only: a handle with a split precision gets
 * HSB_ERR_UNSUPPORTED.  The calls are recorded once into a hipGraph, replayed
 * while n_k, k_frac, ng, out_off and the device pointers stay the same (the
 * graph reads g, tau and T at each replay, so their contents may change);
 * any other change, or hsbuild_set_option, records it again.
 * Workspace: hsbuild_workspace_bytes(h, HSB_MODE_BATCH, n_k, ng). */
int hsbuild_batch(hsbuild_t h, int32_t n_k, const double* k_frac, const int32_t* ng, const int32_t* g,
                  const int64_t* out_off, const double* tau, const void* T, void* H, void* S, void* ws,
                  size_t ws_bytes, void* stream);

/* Stage timing with HIP events recorded on the call's stream, for profiling.
 * hsbuild_set_timing(h, 1) creates an event pool and clears the record;
 * while enabled, each forward entry point (hsbuild_forward, _static,
 * _coefficients, _factored, _real, _hsdla) records events around its
 * HSB_TIMING_STAGES stages (0: coefficients and tables, 1: per-atom T
 * products and, in the split forms, the column scales and the slices or
 * residues of the operands, 2: the H/S contraction kernels, 3: the sum of
 * the stacked-index segments or the residue recombination, empty for the
 * one-pass contractions), for up to HSB_TIMING_CAPACITY calls (later calls
 * are not recorded).  hsbuild_stage_times waits for the recorded events and
 * returns the average milliseconds of each stage over the recorded calls
 * (ms_avg[HSB_TIMING_STAGES]) and their number.  hsbuild_set_timing(h, 0)
 * destroys the pool. */
#define HSB_TIMING_STAGES 4
#define HSB_TIMING_CAPACITY 256
int hsbuild_set_timing(hsbuild_t h, int32_t enable);
int hsbuild_stage_times(hsbuild_t h, double* ms_avg, int32_t* n_calls);

/* Tuning options (performance only).
 * HSB_OPT_TILE_GROUP: order in which the upper-triangle tiles of every
 * contraction are dealt to the compute units: 0 = row-major, g > 0 = super-rows
 * (128 rows; 64 for the factored kernel) taken g at a time, column by column
 * (0..64; default 8, or 4 on a handle with a split precision).  Results are
 * bitwise independent of it.
 * HSB_OPT_HS_WAVES: waves per workgroup of the FP64 contraction, 4 (64 x 32
 * outputs per wave, one wave per SIMD; four real products per complex one) or
 * 8 (32 x 32 per wave, two per SIMD; three real products per complex one, the
 * 3M form; 128 x 128 tiles of 32 x 64 for hsbuild_forward_real, which is
 * real); default 8.  The two complex forms agree to FP64 rounding, not
 * bitwise.  On a handle with a residue form (HSB_SPLIT_CRT*) the option
 * picks the layout of the residue contraction instead (256 x 256 blocks): 4
 * (waves of 128 x 128, one per SIMD; the default there) or 8 (64 x 128, two
 * per SIMD); in HSB_SPLIT_CRT the 4-wave layout keeps its int32 sums
 * unreduced and so runs up to 2048 stages of 64 stacked rows (the real form
 * takes two stages per 64 rows), beyond which the 8-wave layout runs; the
 * 16-bit residue forms run the 8-wave layout only (their default is 8).  All
 * give bitwise the same H and S.
 * HSB_OPT_SPLIT_K: 1 (default) lets the 8-wave FP64 forward run in stream-K
 * form when the upper triangle has fewer than 4 tiles per compute unit and a
 * time model puts it ahead of one pass: the units (128 x 64 tile, 16 stacked
 * rows) are dealt to at most one workgroup per compute unit in equal
 * contiguous shares of at least 256 rows, in a fixed tile order, so small
 * bases fill the GPU; tiles shared between workgroups are summed from their
 * pieces in stacked-row order (the pieces live in the workspace, which
 * hsbuild_workspace_bytes includes).
 * The results agree with the one-pass contraction to FP64 rounding, not
 * bitwise, and repeat bitwise on a device with the same compute-unit count.
 * 0 never splits; k = 2..8 cuts the stacked index into k segments (fewer if
 * it is too short), summed in order.
 * Setting HSB_OPT_TILE_GROUP or HSB_OPT_HS_WAVES drops a captured batch graph
 * (the batch contraction never splits). */
enum { HSB_OPT_TILE_GROUP = 1, HSB_OPT_HS_WAVES = 2, HSB_OPT_SPLIT_K = 3 };
int hsbuild_set_option(hsbuild_t h, int32_t option, int32_t value);
int hsbuild_get_option(hsbuild_t h, int32_t option, int32_t* value);

/* Message of the last error on h (h = NULL: the last hsbuild_create error of
 * this thread).  Valid until the next call on the handle. */
const char* hsbuild_last_error(hsbuild_t h);

/* Host-side evaluation of the device special functions, for checks without a
 * GPU: j_l(x) and j_l'(x) for l = 0..lmax (out arrays of lmax+1 doubles), and
 * pre * i^l conj(Y_lm(K_hat)) for L = 0..(lmax+1)^2-1 (complex128 out). */
int hsbuild_host_bessel(int32_t lmax, double x, double* jl, double* djl);
int hsbuild_host_angular(int32_t lmax, const double kvec[3], double pre, void* out);

/* Matrix-core rate probe, to confirm the peak figures the contraction kernels
 * are measured against: `blocks` workgroups of 4 waves, each wave running 4
 * independent chains of `iters` (a multiple of 16) MFMAs on register operands
 * (HSB_PROBE_FP64: v_mfma_f64_16x16x4f64, the instruction of the FP64
 * contraction; HSB_PROBE_INT8: v_mfma_i32_32x32x32_i8, the instruction of the
 * int8 split contractions, on constant bytes; HSB_PROBE_INT8_RANDOM: the same
 * instruction on hashed bytes in [-120, 120] that change every instruction,
 * like the residue contraction's operands, on which the matrix cores draw more
 * power and may hold a lower clock).  out: device buffer of at least
 * blocks * 256 * 8 bytes (FP64) or blocks * 256 * 4 bytes (INT8, INT8_RANDOM)
 * that receives one value per
 * thread; *ops (host) receives the arithmetic operations the launch executes
 * (2 per multiply-add).  Enqueued on `stream`; the caller times it.  Returns
 * HSB_ERR_ARG or HSB_ERR_WORKSPACE (checked before any device call), or
 * HSB_ERR_DEVICE if the launch fails. */
enum { HSB_PROBE_FP64 = 0, HSB_PROBE_INT8 = 1, HSB_PROBE_INT8_RANDOM = 2 };
int hsbuild_mfma_probe(int32_t kind, int32_t blocks, int32_t iters, void* out, size_t out_bytes, void* stream,
                       double* ops);

#ifdef __cplusplus
}
#endif

#endif /* HSBUILD_H */
