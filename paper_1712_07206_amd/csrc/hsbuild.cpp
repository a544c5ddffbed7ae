// Host side of the hsbuild C-ABI: validation, workspace layout and launch
// sequencing.  No exception crosses the ABI and nothing here allocates device
// memory; the caller owns every device buffer including the workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hs_internal.h"
#include "hsbuild.h"
#include "special.h"

using namespace hsb;

// Workspace of hsbuild_forward_static.  The HIP runtime gives every GPU its own copy of
// this array, alive until the process ends.  On the host the name is only a stand-in for
// the symbol: host code uses the address hipGetSymbolAddress returns for the current
// device (static_scratch below), never the name itself.
static __device__ __align__(256) unsigned char scratch[HSB_STATIC_SCRATCH_BYTES];

struct hsbuild_s {
  int device = 0;
  void* scratch = nullptr;  // this device's copy of `scratch` (device address)
  int n_types = 0, n_atoms = 0, l_max = 0, n_l = 0, max_ng = 0;
  int precision = HSB_FP64, n_slices = 0;
  CrtConsts crt{};  // moduli of the residue form (HSB_SPLIT_CRT)
  int tile_group = 8;  // HSB_OPT_TILE_GROUP
  int hs_waves = 8;    // HSB_OPT_HS_WAVES
  int split_k = 1;     // HSB_OPT_SPLIT_K
  double lattice[9];
  CellArgs cell;              // kfrac filled per call
  TypeConsts* consts = nullptr;  // pinned host copy, source of the per-call upload
  std::string err;
  // stage timing (hsbuild_set_timing)
  std::vector<hipEvent_t> events;  // 4 per recorded call
  int n_timed = 0;
  bool capturing = false;  // no timing events inside a graph capture
  // batch: persistent-kernel grid, captured graph and the arguments it was captured for
  int num_cus = 0;
  hipStream_t cap_stream = nullptr;
  hipStream_t aux[4] = {};            // branches of the batch graph's operand builds
  hipEvent_t fork = nullptr, join[4] = {};
  hipGraphExec_t graph_exec = nullptr;
  hipEvent_t graph_done = nullptr;
  BatchMeta* meta_host = nullptr;  // pinned, source of the graph's metadata upload
  int meta_cap = 0;
  std::vector<double> key_f;
  std::vector<int64_t> key_i;
  // real-symmetric path: pinned sources of the representative upload and its completion event
  int32_t* rep_host = nullptr;
  double* repw_host = nullptr;
  hipEvent_t rep_done = nullptr;
  bool rep_pending = false;
  // BLAS baseline: rocBLAS handle (created on first use) and its device-memory need per basis size
  void* rocblas = nullptr;
  int blas_ng = -1;
  size_t blas_need = 0;
  int eig_ng = -1;  // rocSOLVER's device-memory need of the eigensolve for basis size eig_ng
  size_t eig_need = 0;
};

namespace {

thread_local std::string g_create_error;

int fail(hsbuild_t h, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(hsbuild_t h, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf;
  else g_create_error = buf;
  return code;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Device address of `scratch` on device `dev`, which must be current: looked up once per
// device and kept.  hipSuccess or the lookup's error.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

hipError_t static_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

// Rows of the factored layout: per type with atoms, round16(N_t) phase rows and round16(2 N_L) W0 rows.
int fact_rows(const hsbuild_s& h) {
  int rows = 0;
  for (int t = 0; t < h.n_types; ++t) {
    const int nt = h.cell.type_start[t + 1] - h.cell.type_start[t];
    if (nt > 0) rows += (int)round_up(nt, 16) + (int)round_up(2 * h.n_l, 16);
  }
  return rows;
}

Layout make_layout(const hsbuild_s& h, int ng, int mode) {
  Layout L;
  L.n = ng;
  L.n_pad = (int)round_up(ng, kTileN);
  L.K = 2 * h.n_atoms * h.n_l;
  L.K_pad = stacked_pad(L.K);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t np = (size_t)L.n_pad;
  L.consts = take(sizeof(TypeConsts));
  L.kv = take(np * 4 * sizeof(double));
  L.ang = take((size_t)h.n_l * np * sizeof(double2));
  L.ab = take((size_t)h.n_types * (h.l_max + 1) * np * sizeof(double2));
  if (mode == HSB_MODE_EIGEN) {
    L.eigE = take((size_t)ng * sizeof(double));
    L.blas_bytes = h.eig_ng == ng ? h.eig_need : 0;
    L.blas = take(L.blas_bytes);
    L.end = off;
    return L;
  }
  if (mode == HSB_MODE_HSDLA) {
    const size_t KA = (size_t)h.n_atoms * h.n_l;
    L.hA = take(2 * KA * np * sizeof(double2));  // A stack, then the B stack right after it
    L.hB = L.hA + KA * np * sizeof(double2);
    L.hX = take(KA * np * sizeof(double2));
    L.blas_bytes = h.blas_ng == ng ? h.blas_need : 0;
    L.blas = take(L.blas_bytes);
    L.end = off;
    return L;
  }
  if (mode == HSB_MODE_FACTORED) {
    L.R_f = fact_rows(h);
    L.tau0 = take(4 * sizeof(double));
    L.lamx = take((size_t)L.R_f * sizeof(double));
    L.kind = take((size_t)(L.R_f / 16) * sizeof(int));
    L.X = take((size_t)L.R_f * np * sizeof(double2));
    L.XL = take((size_t)L.R_f * np * sizeof(double2));
    L.Yx = take((size_t)L.R_f * np * sizeof(double2));
    L.TT = take((size_t)h.n_types * tprod_kc(2 * h.n_l) * tprod_mp(2 * h.n_l) * sizeof(double2));
    L.end = off;
    return L;
  }
  if (mode != HSB_MODE_COEFFICIENTS) {
    L.TT = take((size_t)h.n_types * tprod_kc(2 * h.n_l) * tprod_mp(2 * h.n_l) * sizeof(double2));
    L.lam = take((size_t)L.K_pad * sizeof(double));
    L.W = take((size_t)L.K_pad * np * sizeof(double2));
    L.Y = take((size_t)L.K_pad * np * sizeof(double2));
  }
  if ((mode == HSB_MODE_FORWARD || mode == HSB_MODE_REAL) && h.precision == HSB_FP64)
    L.WL = take((size_t)L.K_pad * np * sizeof(double2));
  if (mode == HSB_MODE_FORWARD && h.precision == HSB_FP64 && h.hs_waves == 8 && h.split_k == 1) {
    L.nsh = hs_stream_shares(L.n_pad, L.K_pad, h.num_cus);
    if (L.nsh > 0) {
      L.skH = take(hs_stream_slot_elems(L.nsh) * sizeof(double2));
      L.skS = take(hs_stream_slot_elems(L.nsh) * sizeof(double2));
    }
  } else if (mode == HSB_MODE_FORWARD && h.precision == HSB_FP64 && h.hs_waves == 8 && h.split_k > 1) {
    L.ns = h.split_k;
    while (L.ns > 1 && hs_split_rows(L.K_pad, L.ns) * (L.ns - 1) >= L.K_pad) --L.ns;  // every segment holds rows
    if (L.ns > 1) {
      L.skH = take((size_t)L.ns * np * np * sizeof(double2));
      L.skS = take((size_t)L.ns * np * np * sizeof(double2));
    }
  }
  if ((mode == HSB_MODE_FORWARD || mode == HSB_MODE_REAL) && is_crt(h.precision)) {
    L.K64 = (int)round_up(L.K, kCrtRows);
    L.n_res = crt_cols(ng);
    const size_t nr = (size_t)L.n_res;
    // bytes of one operand's residue planes: bytes, or 16-bit elements
    const size_t planes = (size_t)2 * h.crt.n_mod * L.K64 * nr * (crt_kind(h.precision) ? 2 : 1);
    L.crPart = take((size_t)3 * crt_norm_blocks(L.K) * nr * sizeof(double));
    L.scale = take(3 * nr * sizeof(double));
    L.slL = take(planes);
    L.slS = take(planes);
    L.slY = take(planes);
    L.crRes = take((size_t)h.crt.n_mod * nr * nr * (mode == HSB_MODE_REAL ? 1 : 2));
    L.crResH = take((size_t)h.crt.n_mod * nr * nr * (mode == HSB_MODE_REAL ? 1 : 2));
  } else if ((mode == HSB_MODE_FORWARD && h.precision != HSB_FP64) ||
             (mode == HSB_MODE_REAL && h.precision == HSB_SPLIT_INT8)) {
    L.K_pad2 = (int)round_up(L.K, 32);
    const size_t elem = h.precision == HSB_SPLIT_INT8 ? 1 : 2;       // bytes per slice value
    const size_t planes = (size_t)2 * h.n_slices * np * L.K_pad2 * elem;  // bytes per sliced operand
    L.mx = take(3 * np * sizeof(unsigned long long));
    L.scale = take(3 * np * sizeof(double));
    L.slL = take(planes);
    L.slS = take(planes);
    L.slY = take(planes);
  }
  if (mode == HSB_MODE_REAL) {
    L.rep = take((size_t)h.n_atoms * sizeof(int32_t));
    L.repw = take((size_t)h.n_atoms * sizeof(double));
    L.tau_rep = take((size_t)h.n_atoms * 3 * sizeof(double));
    L.wrow = take((size_t)L.K_pad * sizeof(double));
  }
  if (mode == HSB_MODE_BACKWARD) {
    const size_t M = 2 * (size_t)h.n_l;
    L.PH = take((size_t)L.K_pad * np * sizeof(double2));
    L.PS = take((size_t)L.K_pad * np * sizeof(double2));
    L.Kt = (int)round_up(L.K_pad, 128);
    L.WT = take((size_t)np * L.Kt * sizeof(double2));
    L.gHp = take((size_t)np * np * sizeof(double2));
    L.gSp = take((size_t)np * np * sizeof(double2));
    L.partT = take((size_t)h.n_atoms * M * M * sizeof(double2));
    L.partTau = take((size_t)h.n_atoms * gradtau_blocks(ng) * 3 * sizeof(double));
  }
  L.end = off;
  return L;
}

int check_device(hsbuild_t h) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(h, HSB_ERR_DEVICE, "hipGetDevice failed");
  if (dev != h->device)
    return fail(h, HSB_ERR_DEVICE, "current device %d is not the handle's device %d", dev, h->device);
  return HSB_OK;
}

int check_ws(hsbuild_t h, const Layout& L, void* ws, size_t ws_bytes) {
  if (!ws) return fail(h, HSB_ERR_ARG, "workspace pointer is null");
  if (((uintptr_t)ws) & 255) return fail(h, HSB_ERR_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < L.end)
    return fail(h, HSB_ERR_WORKSPACE, "workspace has %zu bytes, this call needs %zu", ws_bytes, L.end);
  return HSB_OK;
}

int check_ng(hsbuild_t h, int32_t ng) {
  if (ng < 1) return fail(h, HSB_ERR_SHAPE, "ng must be >= 1 (got %d)", ng);
  if (ng > h->max_ng) return fail(h, HSB_ERR_SHAPE, "ng=%d exceeds max_ng=%d given at create", ng, h->max_ng);
  return HSB_OK;
}

int launched(hsbuild_t h, hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(h, HSB_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return HSB_OK;
}

// Records stage boundary `idx` (0..kMarks-1) of the current call when timing is on; the last one
// closes the call's record.
constexpr int kMarks = HSB_TIMING_STAGES + 1;
void mark(hsbuild_t h, int idx, hipStream_t s) {
  if (h->capturing || h->events.empty() || h->n_timed >= HSB_TIMING_CAPACITY) return;
  (void)hipEventRecord(h->events[kMarks * h->n_timed + idx], s);
  if (idx == kMarks - 1) ++h->n_timed;
}

void destroy_events(hsbuild_t h) {
  for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  h->events.clear();
  h->n_timed = 0;
}

// Uploads the type constants and builds K vectors, angular factors and (a, b).
// base: the cell to use instead of the handle's (the representatives of inversion pairs).
// shared: the constants are already in the workspace (batch branches) and are not uploaded again.
int enqueue_tables(hsbuild_t h, const Layout& L, const double k_frac[3], const int32_t* g, char* ws,
                   hipStream_t s, CellArgs& c, const CellArgs* base = nullptr, bool shared = false) {
  c = base ? *base : h->cell;
  for (int i = 0; i < 3; ++i) c.kfrac[i] = k_frac[i];
  TypeConsts* dconsts = (TypeConsts*)(ws + L.consts);
  hipError_t e = hipSuccess;
  if (!shared) e = hipMemcpyAsync(dconsts, h->consts, sizeof(TypeConsts), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return launched(h, e, "upload of type constants");
  e = launch_tables(c, dconsts, L.n, L.n_pad, g, (double2*)(ws + L.ang), (double2*)(ws + L.ab),
                    (double*)(ws + L.kv), s);
  return launched(h, e, "k_tables");
}

// Tables, stacked coefficients W (pad rows zeroed), Y = T W per atom and lam.
// shared: constants and lam are already in the workspace (batch branches).
int enqueue_operands(hsbuild_t h, const Layout& L, const double k_frac[3], const int32_t* g, const double* tau,
                     const void* T, char* ws, hipStream_t s, const CellArgs* base = nullptr, bool shared = false) {
  CellArgs c;
  int rc = enqueue_tables(h, L, k_frac, g, ws, s, c, base, shared);
  if (rc) return rc;
  double2* W = (double2*)(ws + L.W);
  double2* Y = (double2*)(ws + L.Y);
  if (!shared) {  // (the batch prepares lam and T^T once for all k-points)
    rc = launched(h, launch_lambda(c, (const TypeConsts*)(ws + L.consts), L.K_pad, (double*)(ws + L.lam), s),
                  "k_lambda");
    if (!rc) rc = launched(h, launch_tpad((const double2*)T, h->n_types, 2 * h->n_l, (double2*)(ws + L.TT), s),
                           "k_tpad");
    if (rc) return rc;
  }
  rc = launched(h, launch_assemble(c, L.n_pad, (const double2*)(ws + L.ang), (const double2*)(ws + L.ab),
                                   (const double*)(ws + L.kv), tau, W, L.n_pad, L.n_pad, s),
                "k_assemble");
  if (rc) return rc;
  rc = launched(h, launch_zero_rows(W, L.n_pad, L.K, L.K_pad, s), "k_zero_rows");
  if (rc) return rc;
  rc = launched(h, launch_zero_rows(Y, L.n_pad, L.K, L.K_pad, s), "k_zero_rows");
  if (rc) return rc;
  mark(h, 1, s);
  rc = launched(h, launch_tprod(c, (const double2*)(ws + L.TT), W, Y, L.n_pad, s), "k_tprod3m");
  if (!rc && L.WL)  // the FP64 contraction's S operand, lam W
    rc = launched(h, launch_scale_rows(W, (const double*)(ws + L.lam), L.K_pad, L.n_pad, (double2*)(ws + L.WL), s),
                  "k_scale_rows");
  mark(h, 2, s);
  return rc;
}

// The FP64 H/S contraction of the forward (one pass, or in L.ns segments of the stacked index).
// Marks 3 (after the contraction) and 4 (after the segments' sum).
int enqueue_fp64_hs(hsbuild_t h, const Layout& L, char* w, int ng, void* H, void* S, hipStream_t s) {
  const double2 *W = (const double2*)(w + L.W), *WL = (const double2*)(w + L.WL), *Y = (const double2*)(w + L.Y);
  int rc;
  if (L.nsh > 0) {
    double2 *Hp = (double2*)(w + L.skH), *Sp = (double2*)(w + L.skS);
    rc = launched(h, launch_hs_fp64_stream(W, WL, Y, L.K_pad, L.nsh, ng, L.n_pad, (double2*)H, (double2*)S, ng, Hp,
                                           Sp, s),
                  "k_hs_fp64_stream");
    mark(h, 3, s);
    if (!rc)
      rc = launched(h, launch_stream_fixup(L.K_pad, L.nsh, ng, L.n_pad, Hp, Sp, (double2*)H, (double2*)S, ng, s),
                    "k_stream_fixup");
  } else if (L.ns > 1) {
    double2 *Hp = (double2*)(w + L.skH), *Sp = (double2*)(w + L.skS);
    rc = launched(h, launch_hs_fp64_sk(W, WL, Y, L.K_pad, L.ns, ng, L.n_pad, h->tile_group, Hp, Sp, s),
                  "k_hs_fp64_sk");
    mark(h, 3, s);
    if (!rc)
      rc = launched(h, launch_sk_reduce(Hp, Sp, L.ns, ng, L.n_pad, (double2*)H, (double2*)S, ng, s), "k_sk_reduce");
  } else {
    rc = launched(h, launch_hs_fp64(W, WL, Y, (const double*)(w + L.lam), L.K_pad, ng, L.n_pad, h->tile_group,
                                    h->hs_waves, (double2*)H, (double2*)S, ng, s),
                  "k_hs_fp64");
    mark(h, 3, s);
  }
  mark(h, 4, s);
  return rc;
}

// Residue form of the split contraction (complex, or real parts only): column scales, the
// residue planes of W, lam W and Y, then per matrix the residue contraction and the FP64
// recombination.  L.K is the number of stacked rows used (the representatives' in the real case).
int enqueue_crt(hsbuild_t h, const Layout& L, char* w, void* H, void* S, bool real, hipStream_t s) {
  const double2* W = (const double2*)(w + L.W);
  const double2* Y = (const double2*)(w + L.Y);
  const double* lam = (const double*)(w + L.lam);
  double* sc = (double*)(w + L.scale);
  const int ek = crt_kind(h->precision);
  const int QK = (int)round_up(L.K, kCrtRows) / crt_unit_rows(ek);  // 16-byte units per column
  const int nr = L.n_res;
  const CrtConsts& cc = h->crt;
  int rc = launched(h, launch_crt_scales(W, Y, lam, L.K, L.n_pad, nr, cc, (double*)(w + L.crPart), sc, s),
                    "residue scales");
  if (!rc) rc = launched(h, launch_crt_residues(cc, ek, W, lam, 0, L.K, L.n_pad, nr, QK, sc, w + L.slL, s), "residues");
  if (!rc)
    rc = launched(h, launch_crt_residues(cc, ek, W, lam, 1, L.K, L.n_pad, nr, QK, sc + nr, w + L.slS, s), "residues");
  if (!rc)
    rc = launched(h, launch_crt_residues(cc, ek, Y, lam, 0, L.K, L.n_pad, nr, QK, sc + 2 * nr, w + L.slY, s), "residues");
  mark(h, 2, s);  // (again) the operand preparation ends here: the contraction stage starts
  if (!rc)
    rc = launched(h, launch_hs_crt(cc, ek, real, w + L.slL, w + L.slS, QK, L.n, nr, h->tile_group, h->hs_waves,
                                   w + L.crRes, s),
                  "residue contraction (S)");
  if (!rc)
    rc = launched(h, launch_hs_crt(cc, ek, real, w + L.slL, w + L.slY, QK, L.n, nr, h->tile_group, h->hs_waves,
                                   w + L.crResH, s),
                  "residue contraction (H)");
  mark(h, 3, s);
  if (!rc) rc = launched(h, launch_crt_combine(cc, real, w + L.crRes, nr, sc, sc + nr, L.n, S, s), "recombination (S)");
  if (!rc)
    rc = launched(h, launch_crt_combine(cc, real, w + L.crResH, nr, sc, sc + 2 * nr, L.n, H, s), "recombination (H)");
  mark(h, 4, s);
  return rc;
}

// Split-precision contraction: column scales, slices of W, lam W and Y, then S and H.
int enqueue_split(hsbuild_t h, const Layout& L, char* w, double2* H, double2* S, hipStream_t s) {
  if (is_crt(h->precision)) return enqueue_crt(h, L, w, H, S, false, s);
  const double2* W = (const double2*)(w + L.W);
  const double2* Y = (const double2*)(w + L.Y);
  const double* lam = (const double*)(w + L.lam);
  const double* sc = (const double*)(w + L.scale);
  const int QK = L.K_pad2 / (h->precision == HSB_SPLIT_INT8 ? 16 : 8);  // 16-byte units per column
  int rc = launched(h, launch_split_scales(W, Y, lam, L.K, L.n_pad, (unsigned long long*)(w + L.mx), (double*)sc, s),
                    "split scales");
  if (rc) return rc;
  rc = launched(h, launch_split_slices(h->precision, h->n_slices, W, lam, 0, L.K, L.n_pad, QK, sc, w + L.slL, s),
                "split slices");
  if (rc) return rc;
  rc = launched(h, launch_split_slices(h->precision, h->n_slices, W, lam, 1, L.K, L.n_pad, QK, sc + L.n_pad,
                                       w + L.slS, s),
                "split slices");
  if (rc) return rc;
  rc = launched(h, launch_split_slices(h->precision, h->n_slices, Y, lam, 0, L.K, L.n_pad, QK, sc + 2 * L.n_pad,
                                       w + L.slY, s),
                "split slices");
  if (rc) return rc;
  mark(h, 2, s);  // (again) the operand preparation ends here: the contraction stage starts
  rc = launched(h, launch_hs_split(h->precision, h->n_slices, w + L.slL, w + L.slS, sc, sc + L.n_pad, QK, L.n,
                                   L.n_pad, h->tile_group, S, s),
                "split contraction (S)");
  if (rc) return rc;
  rc = launched(h, launch_hs_split(h->precision, h->n_slices, w + L.slL, w + L.slY, sc, sc + 2 * L.n_pad, QK, L.n,
                                   L.n_pad, h->tile_group, H, s),
                "split contraction (H)");
  mark(h, 3, s);  // the slice forms recombine inside the contraction
  mark(h, 4, s);
  return rc;
}

// Real-symmetric int8 split contraction on the representatives' rows (L.K): column scales and
// slices as in the complex form, then S = Re(W^H lam W) and H = Re(W^H Y) into real arrays.
int enqueue_split_real(hsbuild_t h, const Layout& L, char* w, double* H, double* S, hipStream_t s) {
  if (is_crt(h->precision)) return enqueue_crt(h, L, w, H, S, true, s);
  const double2* W = (const double2*)(w + L.W);
  const double2* Y = (const double2*)(w + L.Y);
  const double* lam = (const double*)(w + L.lam);
  const double* sc = (const double*)(w + L.scale);
  const int QK = (int)round_up(L.K, 32) / 16;  // 16-byte units (16 rows of int8) per column
  int rc = launched(h, launch_split_scales(W, Y, lam, L.K, L.n_pad, (unsigned long long*)(w + L.mx), (double*)sc, s),
                    "split scales");
  if (rc) return rc;
  rc = launched(h, launch_split_slices(HSB_SPLIT_INT8, h->n_slices, W, lam, 0, L.K, L.n_pad, QK, sc, w + L.slL, s),
                "split slices");
  if (rc) return rc;
  rc = launched(h, launch_split_slices(HSB_SPLIT_INT8, h->n_slices, W, lam, 1, L.K, L.n_pad, QK, sc + L.n_pad,
                                       w + L.slS, s),
                "split slices");
  if (rc) return rc;
  rc = launched(h, launch_split_slices(HSB_SPLIT_INT8, h->n_slices, Y, lam, 0, L.K, L.n_pad, QK, sc + 2 * L.n_pad,
                                       w + L.slY, s),
                "split slices");
  if (rc) return rc;
  mark(h, 2, s);  // (again) the operand preparation ends here: the contraction stage starts
  rc = launched(h, launch_hs_split8_real(h->n_slices, w + L.slL, w + L.slS, sc, sc + L.n_pad, QK, L.n, L.n_pad,
                                         h->tile_group, S, s),
                "split contraction (real S)");
  if (rc) return rc;
  rc = launched(h, launch_hs_split8_real(h->n_slices, w + L.slL, w + L.slY, sc, sc + 2 * L.n_pad, QK, L.n, L.n_pad,
                                         h->tile_group, H, s),
                "split contraction (real H)");
  mark(h, 3, s);
  mark(h, 4, s);
  return rc;
}

// Operand builds of the k-points run in kBranches parallel graph branches, each with its own tables.
constexpr int kBranches = 4;

struct BatchLayout {
  int K = 0, K_pad = 0, max_n_pad = 0;
  size_t consts = 0, lam = 0, meta = 0, TT = 0, end = 0;
  size_t kv[kBranches] = {}, ang[kBranches] = {}, ab[kBranches] = {};
  std::vector<size_t> W, WL, Y;
  std::vector<int> n_pad;
};

BatchLayout make_batch_layout(const hsbuild_s& h, int n_k, const int32_t* ng) {
  BatchLayout B;
  B.K = 2 * h.n_atoms * h.n_l;
  B.K_pad = stacked_pad(B.K);
  for (int k = 0; k < n_k; ++k) {
    B.n_pad.push_back((int)round_up(ng[k], kTileN));
    B.max_n_pad = std::max(B.max_n_pad, B.n_pad.back());
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t np = (size_t)B.max_n_pad;
  B.consts = take(sizeof(TypeConsts));
  B.lam = take((size_t)B.K_pad * sizeof(double));
  B.TT = take((size_t)h.n_types * tprod_kc(2 * h.n_l) * tprod_mp(2 * h.n_l) * sizeof(double2));
  for (int b = 0; b < kBranches; ++b) {
    B.kv[b] = take(np * 4 * sizeof(double));
    B.ang[b] = take((size_t)h.n_l * np * sizeof(double2));
    B.ab[b] = take((size_t)h.n_types * (h.l_max + 1) * np * sizeof(double2));
  }
  B.meta = take((size_t)n_k * sizeof(BatchMeta));
  for (int k = 0; k < n_k; ++k) {
    B.W.push_back(take((size_t)B.K_pad * B.n_pad[k] * sizeof(double2)));
    B.WL.push_back(take((size_t)B.K_pad * B.n_pad[k] * sizeof(double2)));
    B.Y.push_back(take((size_t)B.K_pad * B.n_pad[k] * sizeof(double2)));
  }
  B.end = off;
  return B;
}

// rocBLAS handle and its device-memory need for basis size ng (both algorithms).
int blas_prepare(hsbuild_t h, int ng) {
  if (int rc = check_device(h)) return rc;  // the rocBLAS handle belongs to the current device
  if (!h->rocblas) {
    std::string err;
    if (hsdla_blas_create(h->device, &h->rocblas, err)) return fail(h, HSB_ERR_DEVICE, "%s", err.c_str());
  }
  if (h->blas_ng == ng) return HSB_OK;
  const int n_pad = (int)round_up(ng, kTileN);
  size_t need = 0;
  for (int alg : {1, 3}) {
    size_t b = 0;
    std::string err;
    if (hsdla_blas_workspace(h->rocblas, alg, h->cell, ng, n_pad, &b, err))
      return fail(h, HSB_ERR_DEVICE, "%s", err.c_str());
    need = std::max(need, b);
  }
  h->blas_ng = ng;
  h->blas_need = need;
  return HSB_OK;
}

// rocBLAS handle and the eigensolve's device-memory need for basis size ng (vectors included).
int eig_prepare(hsbuild_t h, int ng) {
  if (int rc = check_device(h)) return rc;
  if (!h->rocblas) {
    std::string err;
    if (hsdla_blas_create(h->device, &h->rocblas, err)) return fail(h, HSB_ERR_DEVICE, "%s", err.c_str());
  }
  if (h->eig_ng == ng) return HSB_OK;
  size_t need = 0;
  for (bool v : {false, true}) {
    size_t b = 0;
    std::string err;
    if (eig_workspace(h->rocblas, ng, v, &b, err)) return fail(h, HSB_ERR_DEVICE, "%s", err.c_str());
    need = std::max(need, b);
  }
  h->eig_ng = ng;
  h->eig_need = need;
  return HSB_OK;
}

void drop_graph(hsbuild_t h) {
  if (h->graph_exec) {
    if (h->graph_done) (void)hipEventSynchronize(h->graph_done);
    (void)hipGraphExecDestroy(h->graph_exec);
    h->graph_exec = nullptr;
  }
  h->key_f.clear();
  h->key_i.clear();
}

}  // namespace

extern "C" {

int hsbuild_create(const hsb_config* cfg, hsbuild_t* out) {
  g_create_error.clear();
  if (!cfg || !out) return fail(nullptr, HSB_ERR_ARG, "null config or output pointer");
  if (cfg->n_types < 1 || cfg->n_types > HSB_MAX_TYPES)
    return fail(nullptr, HSB_ERR_ARG, "n_types=%d outside [1, %d]", cfg->n_types, HSB_MAX_TYPES);
  if (cfg->n_atoms < 1) return fail(nullptr, HSB_ERR_ARG, "n_atoms=%d must be >= 1", cfg->n_atoms);
  if (cfg->l_max < 0 || cfg->l_max > HSB_MAX_LMAX)
    return fail(nullptr, HSB_ERR_ARG, "l_max=%d outside [0, %d]", cfg->l_max, HSB_MAX_LMAX);
  if (cfg->max_ng < 1) return fail(nullptr, HSB_ERR_ARG, "max_ng=%d must be >= 1", cfg->max_ng);
  if (!cfg->atom_type || !cfg->r_mt || !cfg->radial || !cfg->udot_norm2)
    return fail(nullptr, HSB_ERR_ARG, "null atom_type, r_mt, radial or udot_norm2");
  if (cfg->precision != HSB_FP64 && cfg->precision != HSB_SPLIT_FP16 && cfg->precision != HSB_SPLIT_BF16 &&
      cfg->precision != HSB_SPLIT_INT8 && !is_crt(cfg->precision))
    return fail(nullptr, HSB_ERR_ARG, "unknown precision %d", cfg->precision);
  CrtConsts crt{};
  if (is_crt(cfg->precision)) {
    if (!crt_make_consts(cfg->n_slices, &crt))
      return fail(nullptr, HSB_ERR_ARG, "n_slices=%d (moduli of the residue form) outside [%d, %d]", cfg->n_slices,
                  kCrtMinModuli, kCrtMaxModuli);
  } else if (cfg->precision != HSB_FP64 && (cfg->n_slices < 3 || cfg->n_slices > 6)) {
    return fail(nullptr, HSB_ERR_ARG, "n_slices=%d outside [3, 6]", cfg->n_slices);
  }
  const int n_l = (cfg->l_max + 1) * (cfg->l_max + 1);
  const int64_t K = 2LL * cfg->n_atoms * n_l;
  if (K > (1LL << 30) || (int64_t)cfg->max_ng * (int64_t)round_up(cfg->max_ng, kTileN) > (1LL << 40))
    return fail(nullptr, HSB_ERR_SHAPE, "problem too large");
  // atoms grouped by type
  int type_start[HSB_MAX_TYPES + 1];
  for (int t = 0; t <= cfg->n_types; ++t) type_start[t] = 0;
  int prev = 0;
  for (int a = 0; a < cfg->n_atoms; ++a) {
    const int t = cfg->atom_type[a];
    if (t < 0 || t >= cfg->n_types) return fail(nullptr, HSB_ERR_ARG, "atom %d has type %d", a, t);
    if (t < prev) return fail(nullptr, HSB_ERR_ARG, "atom_type must be non-decreasing (atom %d)", a);
    prev = t;
  }
  {
    int a = 0;
    for (int t = 0; t < cfg->n_types; ++t) {
      type_start[t] = a;
      while (a < cfg->n_atoms && cfg->atom_type[a] == t) ++a;
    }
    type_start[cfg->n_types] = cfg->n_atoms;
  }
  for (int t = 0; t < cfg->n_types; ++t) {
    if (!(cfg->r_mt[t] > 0.0) || !std::isfinite(cfg->r_mt[t]))
      return fail(nullptr, HSB_ERR_ARG, "r_mt[%d] must be positive", t);
    for (int l = 0; l <= cfg->l_max; ++l) {
      const double* r = cfg->radial + ((size_t)t * (cfg->l_max + 1) + l) * 4;
      const double wr = r[0] * r[3] - r[2] * r[1];
      const double scale = std::fabs(r[0] * r[3]) + std::fabs(r[2] * r[1]);
      if (!std::isfinite(wr) || !(std::fabs(wr) >= 1e-12 * scale) || scale == 0.0)
        return fail(nullptr, HSB_ERR_NUMERIC, "radial Wronskian of type %d, l=%d is singular (%g)", t, l, wr);
      const double u2 = cfg->udot_norm2[(size_t)t * (cfg->l_max + 1) + l];
      if (!(u2 >= 0.0) || !std::isfinite(u2))
        return fail(nullptr, HSB_ERR_ARG, "udot_norm2[%d][%d] must be finite and >= 0", t, l);
    }
  }
  // reciprocal basis from the lattice rows
  const double* A = cfg->lattice;
  const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                     A[2] * (A[3] * A[7] - A[4] * A[6]);
  if (!std::isfinite(det) || std::fabs(det) < 1e-9) return fail(nullptr, HSB_ERR_ARG, "degenerate lattice");

  int dev = -1;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(nullptr, HSB_ERR_DEVICE, "no HIP device available");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, HSB_ERR_DEVICE, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);

  void* scratch_dev = nullptr;
  {
    const hipError_t e = static_scratch(dev, &scratch_dev);
    if (e != hipSuccess)
      return fail(nullptr, HSB_ERR_DEVICE, "address of the static scratch on device %d: %s", dev, hipGetErrorString(e));
  }

  hsbuild_s* h = new (std::nothrow) hsbuild_s();
  if (!h) return fail(nullptr, HSB_ERR_ARG, "out of host memory");
  h->scratch = scratch_dev;
  if (hipHostMalloc((void**)&h->consts, sizeof(TypeConsts), hipHostMallocDefault) != hipSuccess) {
    delete h;
    return fail(nullptr, HSB_ERR_DEVICE, "pinned host allocation failed");
  }
  std::memset(h->consts, 0, sizeof(TypeConsts));
  h->device = dev;
  h->num_cus = prop.multiProcessorCount;
  h->n_types = cfg->n_types;
  h->n_atoms = cfg->n_atoms;
  h->l_max = cfg->l_max;
  h->n_l = n_l;
  h->max_ng = cfg->max_ng;
  h->precision = cfg->precision;
  if (cfg->precision != HSB_FP64) h->tile_group = 4;  // measured best for the split contraction
  // residue contraction: waves of 128 x 128 in the byte form (measured best); the 16-bit forms have
  // the 8-wave layout only
  if (is_crt(cfg->precision)) h->hs_waves = crt_kind(cfg->precision) == 0 ? 4 : 8;
  h->n_slices = cfg->n_slices;
  h->crt = crt;
  std::memcpy(h->lattice, cfg->lattice, sizeof h->lattice);
  for (int t = 0; t < cfg->n_types; ++t)
    for (int l = 0; l <= cfg->l_max; ++l) {
      for (int q = 0; q < 4; ++q) h->consts->radial[t][l][q] = cfg->radial[((size_t)t * (cfg->l_max + 1) + l) * 4 + q];
      h->consts->udot2[t][l] = cfg->udot_norm2[(size_t)t * (cfg->l_max + 1) + l];
    }
  CellArgs& c = h->cell;
  std::memset(&c, 0, sizeof c);
  // b_j = 2 pi (A^{-1})^T rows: b_j[i] = 2 pi inv(A)[i][j]
  const double inv[9] = {(A[4] * A[8] - A[5] * A[7]) / det, (A[2] * A[7] - A[1] * A[8]) / det,
                         (A[1] * A[5] - A[2] * A[4]) / det, (A[5] * A[6] - A[3] * A[8]) / det,
                         (A[0] * A[8] - A[2] * A[6]) / det, (A[2] * A[3] - A[0] * A[5]) / det,
                         (A[3] * A[7] - A[4] * A[6]) / det, (A[1] * A[6] - A[0] * A[7]) / det,
                         (A[0] * A[4] - A[1] * A[3]) / det};
  const double two_pi = 6.283185307179586476925286766559;
  for (int j = 0; j < 3; ++j)
    for (int i = 0; i < 3; ++i) c.bvec[3 * j + i] = two_pi * inv[3 * i + j];
  c.pre = 4.0 * 3.14159265358979323846264338327950 / std::sqrt(std::fabs(det));
  c.n_types = cfg->n_types;
  c.n_atoms = cfg->n_atoms;
  c.l_max = cfg->l_max;
  c.n_l = n_l;
  for (int t = 0; t <= cfg->n_types; ++t) c.type_start[t] = type_start[t];
  for (int t = 0; t < cfg->n_types; ++t) c.r_mt[t] = cfg->r_mt[t];
  *out = h;
  return HSB_OK;
}

void hsbuild_destroy(hsbuild_t h) {
  if (!h) return;
  destroy_events(h);
  drop_graph(h);
  if (h->graph_done) (void)hipEventDestroy(h->graph_done);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (int b = 0; b < 4; ++b) {
    if (h->aux[b]) (void)hipStreamDestroy(h->aux[b]);
    if (h->join[b]) (void)hipEventDestroy(h->join[b]);
  }
  if (h->fork) (void)hipEventDestroy(h->fork);
  hsdla_blas_destroy(h->rocblas);
  if (h->rep_done) {
    (void)hipEventSynchronize(h->rep_done);
    (void)hipEventDestroy(h->rep_done);
  }
  if (h->rep_host) (void)hipHostFree(h->rep_host);
  if (h->repw_host) (void)hipHostFree(h->repw_host);
  if (h->meta_host) (void)hipHostFree(h->meta_host);
  if (h->consts) (void)hipHostFree(h->consts);
  delete h;
}

size_t hsbuild_workspace_bytes(hsbuild_t h, int32_t mode, int32_t n_k, const int32_t* ng) {
  if (!h) return 0;
  if (!ng || n_k < 1) {
    fail(h, HSB_ERR_ARG, "ng must point to n_k >= 1 sizes");
    return 0;
  }
  if (mode == HSB_MODE_FORWARD || mode == HSB_MODE_COEFFICIENTS || mode == HSB_MODE_BACKWARD ||
      mode == HSB_MODE_FACTORED || mode == HSB_MODE_HSDLA || mode == HSB_MODE_REAL || mode == HSB_MODE_EIGEN) {
    if (n_k != 1 || check_ng(h, ng[0])) return 0;
    if (mode == HSB_MODE_HSDLA && blas_prepare(h, ng[0])) return 0;
    if (mode == HSB_MODE_EIGEN && eig_prepare(h, ng[0])) return 0;
    return make_layout(*h, ng[0], mode).end;
  }
  if (mode == HSB_MODE_BATCH) {
    for (int k = 0; k < n_k; ++k)
      if (check_ng(h, ng[k])) return 0;
    return make_batch_layout(*h, n_k, ng).end;
  }
  fail(h, HSB_ERR_ARG, "unknown workspace mode %d", mode);
  return 0;
}

int hsbuild_coefficients(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                         void* coef, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  if (!k_frac || !g || !tau || !coef) return fail(h, HSB_ERR_ARG, "null k_frac, g, tau or coef");
  int rc = check_ng(h, ng);
  if (rc) return rc;
  const Layout L = make_layout(*h, ng, HSB_MODE_COEFFICIENTS);
  if ((rc = check_ws(h, L, ws, ws_bytes))) return rc;
  if ((rc = check_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  CellArgs c;
  if ((rc = enqueue_tables(h, L, k_frac, g, (char*)ws, s, c))) return rc;
  char* w = (char*)ws;
  return launched(h, launch_assemble(c, L.n_pad, (const double2*)(w + L.ang), (const double2*)(w + L.ab),
                                     (const double*)(w + L.kv), tau, (double2*)coef, ng, ng, s),
                  "k_assemble");
}

}  // extern "C"

namespace {

// Body of hsbuild_forward and hsbuild_forward_static once the arguments and the
// workspace `w` (L.end bytes) have been checked.
int forward_enqueue(hsbuild_t h, const Layout& L, const double k_frac[3], int32_t ng, const int32_t* g,
                    const double* tau, const void* T, void* H, void* S, char* w, hipStream_t s) {
  int rc;
  mark(h, 0, s);
  if ((rc = enqueue_operands(h, L, k_frac, g, tau, T, w, s))) return rc;
  if (h->precision == HSB_FP64) {
    rc = enqueue_fp64_hs(h, L, w, ng, H, S, s);  // marks 3 and 4
  } else {
    rc = enqueue_split(h, L, w, (double2*)H, (double2*)S, s);  // marks 2 (again), 3 and 4
  }
  return rc;
}

}  // namespace

extern "C" {

int hsbuild_forward(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                    const void* T, void* H, void* S, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  if (!k_frac || !g || !tau || !T || !H || !S) return fail(h, HSB_ERR_ARG, "null k_frac, g, tau, T, H or S");
  if (H == S) return fail(h, HSB_ERR_ARG, "H and S must be distinct buffers");
  int rc = check_ng(h, ng);
  if (rc) return rc;
  const Layout L = make_layout(*h, ng, HSB_MODE_FORWARD);
  if ((rc = check_ws(h, L, ws, ws_bytes))) return rc;
  if ((rc = check_device(h))) return rc;
  return forward_enqueue(h, L, k_frac, ng, g, tau, T, H, S, (char*)ws, (hipStream_t)stream);
}

int hsbuild_forward_static(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                           const void* T, void* H, void* S, void* stream) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  if (!k_frac || !g || !tau || !T || !H || !S) return fail(h, HSB_ERR_ARG, "null k_frac, g, tau, T, H or S");
  if (H == S) return fail(h, HSB_ERR_ARG, "H and S must be distinct buffers");
  int rc = check_ng(h, ng);
  if (rc) return rc;
  const Layout L = make_layout(*h, ng, HSB_MODE_FORWARD);
  if (L.end > HSB_STATIC_SCRATCH_BYTES)
    return fail(h, HSB_ERR_WORKSPACE,
                "ng=%d needs %zu bytes of workspace, the static scratch holds %zu; use hsbuild_forward with a "
                "caller workspace",
                ng, L.end, (size_t)HSB_STATIC_SCRATCH_BYTES);
  if ((rc = check_device(h))) return rc;
  if (!h->scratch) return fail(h, HSB_ERR_DEVICE, "no static scratch address for device %d", h->device);
  return forward_enqueue(h, L, k_frac, ng, g, tau, T, H, S, (char*)h->scratch, (hipStream_t)stream);
}

int hsbuild_forward_factored(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                             const void* T, void* H, void* S, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  if (!k_frac || !g || !tau || !T || !H || !S) return fail(h, HSB_ERR_ARG, "null k_frac, g, tau, T, H or S");
  if (H == S) return fail(h, HSB_ERR_ARG, "H and S must be distinct buffers");
  int rc = check_ng(h, ng);
  if (rc) return rc;
  const Layout L = make_layout(*h, ng, HSB_MODE_FACTORED);
  if ((rc = check_ws(h, L, ws, ws_bytes))) return rc;
  if ((rc = check_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const int64_t np = L.n_pad;
  const int M = 2 * h->n_l, Mp = (int)round_up(M, 16);
  double2* X = (double2*)(w + L.X);
  double2* XL = (double2*)(w + L.XL);
  double2* Yx = (double2*)(w + L.Yx);
  mark(h, 0, s);
  CellArgs c;
  if ((rc = enqueue_tables(h, L, k_frac, g, w, s, c))) return rc;
  const TypeConsts* dconsts = (const TypeConsts*)(w + L.consts);
  rc = launched(h, launch_fact_rows(c, dconsts, L.R_f, (double*)(w + L.lamx), (int*)(w + L.kind), s), "k_fact_rows");
  if (rc) return rc;
  // origin of every type (phase 1): two zero double2 = four zero doubles
  if ((rc = launched(h, launch_zero_rows((double2*)(w + L.tau0), 2, 0, 1, s), "k_zero_rows"))) return rc;
  int base = 0;
  for (int t = 0; t < h->n_types; ++t) {
    const int a0 = c.type_start[t], nt = c.type_start[t + 1] - a0;
    if (nt == 0) continue;
    const int Ep = (int)round_up(nt, 16), rw = base + Ep;
    // phase rows of the type's atoms, zero pad rows; Yx is zero on the whole phase block
    rc = launched(h, launch_phases(nt, L.n_pad, (const double*)(w + L.kv), tau + 3 * a0, X + (int64_t)base * np, s),
                  "k_phases");
    if (!rc) rc = launched(h, launch_zero_rows(X, np, base + nt, rw, s), "k_zero_rows");
    if (!rc) rc = launched(h, launch_zero_rows(Yx, np, base, rw, s), "k_zero_rows");
    // W0_t: the type's coefficients at the origin (one-atom cell of type t), zero pad rows
    CellArgs c1 = c;
    c1.n_types = 1;
    c1.n_atoms = 1;
    c1.type_start[0] = 0;
    c1.type_start[1] = 1;
    c1.r_mt[0] = c.r_mt[t];
    const double2* ab_t = (const double2*)(w + L.ab) + (int64_t)t * (h->l_max + 1) * np;
    if (!rc)
      rc = launched(h, launch_assemble(c1, L.n_pad, (const double2*)(w + L.ang), ab_t, (const double*)(w + L.kv),
                                       (const double*)(w + L.tau0), X + (int64_t)rw * np, np, L.n_pad, s),
                    "k_assemble");
    if (!rc) rc = launched(h, launch_zero_rows(X, np, rw + M, rw + Mp, s), "k_zero_rows");
    if (!rc) rc = launched(h, launch_zero_rows(Yx, np, rw + M, rw + Mp, s), "k_zero_rows");
    if (rc) return rc;
    base = rw + Mp;
  }
  mark(h, 1, s);
  rc = launched(h, launch_tpad((const double2*)T, h->n_types, M, (double2*)(w + L.TT), s), "k_tpad");
  if (rc) return rc;
  base = 0;
  for (int t = 0; t < h->n_types; ++t) {
    const int nt = c.type_start[t + 1] - c.type_start[t];
    if (nt == 0) continue;
    const int rw = base + (int)round_up(nt, 16);
    CellArgs c1 = c;
    c1.n_types = 1;
    c1.n_atoms = 1;
    c1.type_start[0] = 0;
    c1.type_start[1] = 1;
    rc = launched(h, launch_tprod(c1, (const double2*)(w + L.TT) + (int64_t)t * tprod_kc(M) * tprod_mp(M),
                                  X + (int64_t)rw * np, Yx + (int64_t)rw * np, L.n_pad, s),
                  "k_tprod3m");
    if (rc) return rc;
    base = rw + Mp;
  }
  rc = launched(h, launch_scale_rows(X, (const double*)(w + L.lamx), L.R_f, L.n_pad, XL, s), "k_scale_rows");
  if (rc) return rc;
  mark(h, 2, s);
  rc = launched(h, launch_hs_fact(X, XL, Yx, (const int*)(w + L.kind), L.R_f / 16, ng, L.n_pad, h->tile_group,
                                  (double2*)H, (double2*)S, ng, s),
                "k_hs_fact");
  mark(h, 3, s);
  mark(h, 4, s);
  return rc;
}

int hsbuild_forward_real(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                         const int32_t* partner, const void* T, double* H, double* S, void* ws, size_t ws_bytes,
                         void* stream) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  if (!k_frac || !g || !tau || !partner || !T || !H || !S)
    return fail(h, HSB_ERR_ARG, "null k_frac, g, tau, partner, T, H or S");
  if (H == S) return fail(h, HSB_ERR_ARG, "H and S must be distinct buffers");
  if (h->precision != HSB_FP64 && h->precision != HSB_SPLIT_INT8 && !is_crt(h->precision))
    return fail(h, HSB_ERR_UNSUPPORTED,
                "the real-symmetric build has FP64, int8 slice and residue forms only (no BF16/FP16)");
  int rc = check_ng(h, ng);
  if (rc) return rc;
  // representatives: the lower index of each inversion pair (weight 2), atoms paired with themselves (weight 1)
  const CellArgs& cell = h->cell;
  auto type_of = [&](int a) {
    int t = 0;
    while (t + 1 < cell.n_types && a >= cell.type_start[t + 1]) ++t;
    return t;
  };
  std::vector<int32_t> rep;
  std::vector<double> wt;
  CellArgs crep = cell;
  for (int t = 0; t <= HSB_MAX_TYPES; ++t) crep.type_start[t] = 0;
  for (int a = 0; a < h->n_atoms; ++a) {
    const int p = partner[a];
    if (p < 0 || p >= h->n_atoms || partner[p] != a)
      return fail(h, HSB_ERR_ARG, "partner is not an involution at atom %d", a);
    if (type_of(p) != type_of(a)) return fail(h, HSB_ERR_ARG, "atoms %d and %d are paired but differ in type", a, p);
    if (p >= a) {
      rep.push_back(a);
      wt.push_back(p == a ? 1.0 : 2.0);
      crep.type_start[type_of(a) + 1] += 1;
    }
  }
  for (int t = 0; t < cell.n_types; ++t) crep.type_start[t + 1] += crep.type_start[t];
  const int n_rep = (int)rep.size();
  crep.n_atoms = n_rep;
  const Layout L = make_layout(*h, ng, HSB_MODE_REAL);
  if ((rc = check_ws(h, L, ws, ws_bytes))) return rc;
  if ((rc = check_device(h))) return rc;
  Layout Lr = L;  // the stacked rows of the representatives only
  Lr.K = 2 * n_rep * h->n_l;
  Lr.K_pad = stacked_pad(Lr.K);
  Lr.WL = 0;  // lam W is formed below, after the pair weights are folded into lam
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  // upload the representatives from pinned memory (after the previous upload has been consumed)
  if (!h->rep_host) {
    if (hipHostMalloc((void**)&h->rep_host, sizeof(int32_t) * h->n_atoms, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h->repw_host, sizeof(double) * h->n_atoms, hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&h->rep_done, hipEventDisableTiming) != hipSuccess)
      return fail(h, HSB_ERR_DEVICE, "pinned buffer or event for the representatives");
  }
  if (h->rep_pending && hipEventSynchronize(h->rep_done) != hipSuccess)
    return fail(h, HSB_ERR_DEVICE, "hipEventSynchronize failed");
  h->rep_pending = false;
  std::memcpy(h->rep_host, rep.data(), sizeof(int32_t) * n_rep);
  std::memcpy(h->repw_host, wt.data(), sizeof(double) * n_rep);
  mark(h, 0, s);
  hipError_t e = hipMemcpyAsync(w + L.rep, h->rep_host, sizeof(int32_t) * n_rep, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(w + L.repw, h->repw_host, sizeof(double) * n_rep, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(h->rep_done, s);
  if (e != hipSuccess) return launched(h, e, "upload of the representatives");
  h->rep_pending = true;
  const int rows = 2 * h->n_l;
  double* tau_rep = (double*)(w + L.tau_rep);
  rc = launched(h, launch_rep_setup(tau, (const int*)(w + L.rep), (const double*)(w + L.repw), n_rep, rows, 0,
                                    tau_rep, nullptr, nullptr, s),
                "k_rep_setup");
  if (rc) return rc;
  if ((rc = enqueue_operands(h, Lr, k_frac, g, tau_rep, T, w, s, &crep))) return rc;
  // weights: lam *= w per row (S), Y rows times w (H)
  double* lam = (double*)(w + L.lam);
  double* wrow = (double*)(w + L.wrow);
  double2* Y = (double2*)(w + L.Y);
  rc = launched(h, launch_rep_setup(tau, (const int*)(w + L.rep), (const double*)(w + L.repw), n_rep, rows, Lr.K_pad,
                                    tau_rep, wrow, lam, s),
                "k_rep_setup");
  if (!rc) rc = launched(h, launch_scale_rows(Y, wrow, Lr.K_pad, L.n_pad, Y, s), "k_scale_rows");
  if (!rc && (h->precision == HSB_SPLIT_INT8 || is_crt(h->precision))) {
    rc = enqueue_split_real(h, Lr, w, H, S, s);
  } else if (!rc) {
    double2* WL = (double2*)(w + L.WL);  // S's right operand, lam W (lam with the pair weights)
    rc = launched(h, launch_scale_rows((const double2*)(w + L.W), lam, Lr.K_pad, L.n_pad, WL, s), "k_scale_rows");
    if (!rc)
      rc = launched(h, launch_hs_fp64_real((const double2*)(w + L.W), WL, Y, lam, Lr.K_pad, ng, L.n_pad,
                                           h->tile_group, h->hs_waves, H, S, ng, s),
                    "k_hs_fp64 (real)");
    mark(h, 3, s);
    mark(h, 4, s);
  }
  return rc;
}

int hsbuild_eigensolve(hsbuild_t h, int32_t ng, void* H, void* S, double* w, int32_t vectors, int32_t* info, void* ws,
                       size_t ws_bytes, void* stream) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  if (!H || !S || !w || !info) return fail(h, HSB_ERR_ARG, "null H, S, w or info");
  if (H == S) return fail(h, HSB_ERR_ARG, "H and S must be distinct buffers");
  if (vectors != 0 && vectors != 1) return fail(h, HSB_ERR_ARG, "vectors must be 0 or 1 (got %d)", vectors);
  int rc = check_ng(h, ng);
  if (rc) return rc;
  if ((rc = eig_prepare(h, ng))) return rc;
  const Layout L = make_layout(*h, ng, HSB_MODE_EIGEN);
  if ((rc = check_ws(h, L, ws, ws_bytes))) return rc;
  hipStream_t s = (hipStream_t)stream;
  char* wsp = (char*)ws;
  std::string err;
  if (hsdla_blas_bind(h->rocblas, L.blas_bytes ? wsp + L.blas : nullptr, L.blas_bytes, s, err))
    return fail(h, HSB_ERR_DEVICE, "%s", err.c_str());
  if (eig_enqueue(h->rocblas, ng, (double2*)H, (double2*)S, w, (double*)(wsp + L.eigE), (int*)info, vectors != 0,
                  err))
    return fail(h, HSB_ERR_DEVICE, "%s", err.c_str());
  if (vectors) return launched(h, launch_conj((double2*)H, (int64_t)ng * ng, s), "k_conj");
  return HSB_OK;
}

int hsbuild_forward_hsdla(hsbuild_t h, int32_t algorithm, const double k_frac[3], int32_t ng, const int32_t* g,
                          const double* tau, const void* T, void* H, void* S, void* ws, size_t ws_bytes,
                          void* stream) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  if (algorithm != 1 && algorithm != 3) return fail(h, HSB_ERR_ARG, "algorithm must be 1 or 3 (got %d)", algorithm);
  if (!k_frac || !g || !tau || !T || !H || !S) return fail(h, HSB_ERR_ARG, "null k_frac, g, tau, T, H or S");
  if (H == S) return fail(h, HSB_ERR_ARG, "H and S must be distinct buffers");
  int rc = check_ng(h, ng);
  if (rc) return rc;
  if ((rc = check_device(h))) return rc;
  if ((rc = blas_prepare(h, ng))) return rc;
  const Layout L = make_layout(*h, ng, HSB_MODE_HSDLA);
  if ((rc = check_ws(h, L, ws, ws_bytes))) return rc;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  std::string err;
  if (hsdla_blas_bind(h->rocblas, L.blas_bytes ? w + L.blas : nullptr, L.blas_bytes, s, err))
    return fail(h, HSB_ERR_DEVICE, "%s", err.c_str());
  mark(h, 0, s);
  CellArgs c;
  if ((rc = enqueue_tables(h, L, k_frac, g, w, s, c))) return rc;
  // A stack (rows (atom, L)) followed by the B stack
  rc = launched(h, launch_assemble_split(c, L.n_pad, (const double2*)(w + L.ang), (const double2*)(w + L.ab),
                                         (const double*)(w + L.kv), tau, (double2*)(w + L.hA), L.n_pad, L.n_pad, s),
                "k_assemble");
  if (rc) return rc;
  mark(h, 1, s);
  mark(h, 2, s);
  if (hsdla_blas_enqueue(h->rocblas, algorithm, c, (const TypeConsts*)(w + L.consts), ng, L.n_pad, (const double2*)T,
                         (const double2*)(w + L.hA), (const double2*)(w + L.hB), (double2*)(w + L.hX), (double2*)H,
                         (double2*)S, s, false, err))
    return fail(h, HSB_ERR_DEVICE, "%s", err.c_str());
  mark(h, 3, s);
  mark(h, 4, s);
  return HSB_OK;
}

int hsbuild_forward_coefficients(hsbuild_t h, int32_t ng, const void* coef, const void* T, void* H, void* S,
                                 void* ws, size_t ws_bytes, void* stream) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  if (!coef || !T || !H || !S) return fail(h, HSB_ERR_ARG, "null coef, T, H or S");
  if (H == S) return fail(h, HSB_ERR_ARG, "H and S must be distinct buffers");
  int rc = check_ng(h, ng);
  if (rc) return rc;
  const Layout L = make_layout(*h, ng, HSB_MODE_FORWARD);
  if ((rc = check_ws(h, L, ws, ws_bytes))) return rc;
  if ((rc = check_device(h))) return rc;
  if (L.K > 65535 * 64) return fail(h, HSB_ERR_SHAPE, "stacked width too large for this entry point");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  CellArgs c = h->cell;
  double2* W = (double2*)(w + L.W);
  double2* Y = (double2*)(w + L.Y);
  mark(h, 0, s);
  hipError_t e = hipMemcpyAsync(w + L.consts, h->consts, sizeof(TypeConsts), hipMemcpyHostToDevice, s);
  if ((rc = launched(h, e, "upload of type constants"))) return rc;
  if ((rc = launched(h, launch_lambda(c, (const TypeConsts*)(w + L.consts), L.K_pad, (double*)(w + L.lam), s),
                     "k_lambda")))
    return rc;
  for (int r0 = 0; r0 < L.K; r0 += 65535) {  // grid.y limit
    const int rows = std::min(65535, L.K - r0);
    if ((rc = launched(h, launch_pack_rows((const double2*)coef + (int64_t)r0 * ng, ng, rows,
                                           W + (int64_t)r0 * L.n_pad, L.n_pad, s),
                       "k_pack_rows")))
      return rc;
  }
  if ((rc = launched(h, launch_zero_rows(W, L.n_pad, L.K, L.K_pad, s), "k_zero_rows"))) return rc;
  if ((rc = launched(h, launch_zero_rows(Y, L.n_pad, L.K, L.K_pad, s), "k_zero_rows"))) return rc;
  mark(h, 1, s);
  if ((rc = launched(h, launch_tpad((const double2*)T, h->n_types, 2 * h->n_l, (double2*)(w + L.TT), s), "k_tpad")))
    return rc;
  if ((rc = launched(h, launch_tprod(c, (const double2*)(w + L.TT), W, Y, L.n_pad, s), "k_tprod3m"))) return rc;
  if (h->precision == HSB_FP64) {
    double2* WL = (double2*)(w + L.WL);
    if ((rc = launched(h, launch_scale_rows(W, (const double*)(w + L.lam), L.K_pad, L.n_pad, WL, s), "k_scale_rows")))
      return rc;
    mark(h, 2, s);
    return enqueue_fp64_hs(h, L, w, ng, H, S, s);
  }
  mark(h, 2, s);
  return enqueue_split(h, L, w, (double2*)H, (double2*)S, s);
}

int hsbuild_backward(hsbuild_t h, const double k_frac[3], int32_t ng, const int32_t* g, const double* tau,
                     const void* T, const void* gH, const void* gS, void* gT, double* gtau, void* ws,
                     size_t ws_bytes, void* stream) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  if (!k_frac || !g || !tau || !T || !gH || !gS || !gT || !gtau)
    return fail(h, HSB_ERR_ARG, "null k_frac, g, tau, T, gH, gS, gT or gtau");
  int rc = check_ng(h, ng);
  if (rc) return rc;
  const Layout L = make_layout(*h, ng, HSB_MODE_BACKWARD);
  if ((rc = check_ws(h, L, ws, ws_bytes))) return rc;
  if ((rc = check_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  if ((rc = enqueue_operands(h, L, k_frac, g, tau, T, w, s))) return rc;
  CellArgs c = h->cell;
  const double2* W = (const double2*)(w + L.W);
  double2* PH = (double2*)(w + L.PH);
  double2* PS = (double2*)(w + L.PS);
  // P_H = W gH, P_S = W gS in the 3M form, from W^T and zero-padded gH, gS
  double2* WT = (double2*)(w + L.WT);
  double2* gHp = (double2*)(w + L.gHp);
  double2* gSp = (double2*)(w + L.gSp);
  rc = launched(h, launch_transpose(W, L.K_pad, L.n_pad, L.Kt, WT, s), "k_transpose");
  if (!rc) rc = launched(h, launch_pad_square((const double2*)gH, ng, L.n_pad, gHp, s), "k_pad_square");
  if (!rc) rc = launched(h, launch_pad_square((const double2*)gS, ng, L.n_pad, gSp, s), "k_pad_square");
  if (!rc) rc = launched(h, launch_pgemm3m(WT, gSp, gHp, L.Kt, L.K_pad, L.n_pad, PH, PS, s), "k_pgemm3m");
  if (rc) return rc;
  rc = launched(h, launch_gradT(c, PH, W, L.n_pad, (double2*)(w + L.partT), (double2*)gT, s), "k_gradT");
  if (rc) return rc;
  return launched(h, launch_gradtau(c, PH, PS, (const double2*)(w + L.Y), W, (const double*)(w + L.lam),
                                    (const double*)(w + L.kv), ng, L.n_pad, (double*)(w + L.partTau), gtau, s),
                  "k_gradtau");
}

int hsbuild_batch(hsbuild_t h, int32_t n_k, const double* k_frac, const int32_t* ng, const int32_t* g,
                  const int64_t* out_off, const double* tau, const void* T, void* H, void* S, void* ws,
                  size_t ws_bytes, void* stream) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  if (n_k < 1) return fail(h, HSB_ERR_ARG, "n_k must be >= 1 (got %d)", n_k);
  if (!k_frac || !ng || !g || !out_off || !tau || !T || !H || !S)
    return fail(h, HSB_ERR_ARG, "null k_frac, ng, g, out_off, tau, T, H or S");
  if (H == S) return fail(h, HSB_ERR_ARG, "H and S must be distinct buffers");
  if (h->precision != HSB_FP64)
    return fail(h, HSB_ERR_UNSUPPORTED, "batch runs the FP64 contraction only");
  int rc;
  for (int k = 0; k < n_k; ++k)
    if ((rc = check_ng(h, ng[k]))) return rc;
  {  // output blocks must not overlap
    std::vector<std::pair<int64_t, int64_t>> blocks;
    for (int k = 0; k < n_k; ++k) {
      if (out_off[k] < 0) return fail(h, HSB_ERR_ARG, "out_off[%d] is negative", k);
      blocks.push_back({out_off[k], out_off[k] + (int64_t)ng[k] * ng[k]});
    }
    std::sort(blocks.begin(), blocks.end());
    for (size_t i = 1; i < blocks.size(); ++i)
      if (blocks[i].first < blocks[i - 1].second) return fail(h, HSB_ERR_SHAPE, "output blocks overlap");
  }
  const BatchLayout B = make_batch_layout(*h, n_k, ng);
  if (!ws) return fail(h, HSB_ERR_ARG, "workspace pointer is null");
  if (((uintptr_t)ws) & 255) return fail(h, HSB_ERR_ARG, "workspace must be 256-byte aligned");
  if (ws_bytes < B.end)
    return fail(h, HSB_ERR_WORKSPACE, "workspace has %zu bytes, this call needs %zu", ws_bytes, B.end);
  if ((rc = check_device(h))) return rc;
  hipStream_t s = (hipStream_t)stream;

  // the graph is reused when every argument matches the call it was captured for
  std::vector<double> kf(k_frac, k_frac + 3 * (size_t)n_k);
  std::vector<int64_t> ki = {n_k, (int64_t)(uintptr_t)g, (int64_t)(uintptr_t)tau, (int64_t)(uintptr_t)T,
                             (int64_t)(uintptr_t)H, (int64_t)(uintptr_t)S, (int64_t)(uintptr_t)ws,
                             (int64_t)ws_bytes};
  for (int k = 0; k < n_k; ++k) {
    ki.push_back(ng[k]);
    ki.push_back(out_off[k]);
  }
  if (!(h->graph_exec && kf == h->key_f && ki == h->key_i)) {
    drop_graph(h);
    if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess)
      return fail(h, HSB_ERR_DEVICE, "hipStreamCreateWithFlags failed");
    if (!h->graph_done && hipEventCreateWithFlags(&h->graph_done, hipEventDisableTiming) != hipSuccess)
      return fail(h, HSB_ERR_DEVICE, "hipEventCreate failed");
    if (n_k > h->meta_cap) {
      if (h->meta_host) (void)hipHostFree(h->meta_host);
      h->meta_host = nullptr;
      h->meta_cap = 0;
      if (hipHostMalloc((void**)&h->meta_host, sizeof(BatchMeta) * n_k, hipHostMallocDefault) != hipSuccess)
        return fail(h, HSB_ERR_DEVICE, "pinned host allocation failed");
      h->meta_cap = n_k;
    }
    int total = 0;
    for (int k = 0; k < n_k; ++k) {
      BatchMeta& m = h->meta_host[k];
      m.w_off = (int64_t)(B.W[k] / sizeof(double2));
      m.wl_off = (int64_t)(B.WL[k] / sizeof(double2));
      m.y_off = (int64_t)(B.Y[k] / sizeof(double2));
      m.out_off = out_off[k];
      m.n = ng[k];
      m.n_pad = B.n_pad[k];
      m.nbr = B.n_pad[k] / kTileN;
      m.tile_start = total;
      total += hs_tiles(B.n_pad[k]);
    }
    for (int b = 0; b < kBranches; ++b) {
      if (!h->aux[b] && hipStreamCreateWithFlags(&h->aux[b], hipStreamNonBlocking) != hipSuccess)
        return fail(h, HSB_ERR_DEVICE, "hipStreamCreateWithFlags failed");
      if (!h->join[b] && hipEventCreateWithFlags(&h->join[b], hipEventDisableTiming) != hipSuccess)
        return fail(h, HSB_ERR_DEVICE, "hipEventCreate failed");
    }
    if (!h->fork && hipEventCreateWithFlags(&h->fork, hipEventDisableTiming) != hipSuccess)
      return fail(h, HSB_ERR_DEVICE, "hipEventCreate failed");
    hipStream_t cs = h->cap_stream;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess)
      return fail(h, HSB_ERR_DEVICE, "hipStreamBeginCapture failed");
    char* w = (char*)ws;
    rc = HSB_OK;
    h->capturing = true;
    // shared inputs once: type constants and lam; then the k-points' operands in parallel branches
    hipError_t ef = hipMemcpyAsync(w + B.consts, h->consts, sizeof(TypeConsts), hipMemcpyHostToDevice, cs);
    if (ef == hipSuccess) ef = launch_lambda(h->cell, (const TypeConsts*)(w + B.consts), B.K_pad, (double*)(w + B.lam), cs);
    if (ef == hipSuccess) ef = launch_tpad((const double2*)T, h->n_types, 2 * h->n_l, (double2*)(w + B.TT), cs);
    if (ef == hipSuccess) ef = hipEventRecord(h->fork, cs);
    for (int b = 0; b < kBranches && ef == hipSuccess; ++b) ef = hipStreamWaitEvent(h->aux[b], h->fork, 0);
    if (ef != hipSuccess) rc = launched(h, ef, "batch graph fork");
    std::vector<int64_t> g_rows(n_k, 0);
    for (int k = 1; k < n_k; ++k) g_rows[k] = g_rows[k - 1] + ng[k - 1];
    for (int k = 0; k < n_k && rc == HSB_OK; ++k) {
      const int b = k % kBranches;
      Layout L;
      L.n = ng[k];
      L.n_pad = B.n_pad[k];
      L.K = B.K;
      L.K_pad = B.K_pad;
      L.consts = B.consts;
      L.lam = B.lam;
      L.TT = B.TT;
      L.kv = B.kv[b];
      L.ang = B.ang[b];
      L.ab = B.ab[b];
      L.W = B.W[k];
      L.WL = B.WL[k];
      L.Y = B.Y[k];
      rc = enqueue_operands(h, L, k_frac + 3 * k, g + 3 * g_rows[k], tau, T, w, h->aux[b], nullptr, true);
    }
    for (int b = 0; b < kBranches; ++b) {  // join every branch back, also after an error
      hipError_t ej = hipEventRecord(h->join[b], h->aux[b]);
      if (ej == hipSuccess) ej = hipStreamWaitEvent(cs, h->join[b], 0);
      if (ej != hipSuccess && rc == HSB_OK) rc = launched(h, ej, "batch graph join");
    }
    if (rc == HSB_OK) {
      hipError_t e = hipMemcpyAsync(w + B.meta, h->meta_host, sizeof(BatchMeta) * n_k, hipMemcpyHostToDevice, cs);
      if (e == hipSuccess) {
        const int grid = std::max(8, (h->num_cus / 8) * 8);  // one workgroup per CU, a multiple of 8
        e = launch_hs_fp64_batch((const double2*)w, (const double*)(w + B.lam), B.K_pad,
                                 (const BatchMeta*)(w + B.meta), n_k, total, grid, h->tile_group, h->hs_waves,
                                 (double2*)H, (double2*)S, cs);
      }
      if (e != hipSuccess) rc = launched(h, e, "batched contraction");
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    h->capturing = false;
    if (rc != HSB_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (ec != hipSuccess || !graph) return fail(h, HSB_ERR_DEVICE, "hipStreamEndCapture failed");
    const hipError_t ei = hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      h->graph_exec = nullptr;
      return fail(h, HSB_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    }
    h->key_f = kf;
    h->key_i = ki;
  }
  hipError_t e = hipGraphLaunch(h->graph_exec, s);
  if (e != hipSuccess) return launched(h, e, "hipGraphLaunch");
  return launched(h, hipEventRecord(h->graph_done, s), "hipEventRecord");
}

int hsbuild_set_timing(hsbuild_t h, int32_t enable) {
  if (!h) return HSB_ERR_ARG;
  destroy_events(h);
  if (!enable) return HSB_OK;
  h->events.resize(kMarks * HSB_TIMING_CAPACITY);
  for (size_t i = 0; i < h->events.size(); ++i) {
    if (hipEventCreate(&h->events[i]) != hipSuccess) {
      h->events.resize(i);
      destroy_events(h);
      return fail(h, HSB_ERR_DEVICE, "hipEventCreate failed");
    }
  }
  return HSB_OK;
}

int hsbuild_stage_times(hsbuild_t h, double* ms_avg, int32_t* n_calls) {
  if (!h || !ms_avg || !n_calls) return HSB_ERR_ARG;
  if (h->events.empty()) return fail(h, HSB_ERR_ARG, "timing is not enabled");
  double acc[HSB_TIMING_STAGES] = {};
  for (int c = 0; c < h->n_timed; ++c) {
    if (hipEventSynchronize(h->events[kMarks * c + kMarks - 1]) != hipSuccess)
      return fail(h, HSB_ERR_DEVICE, "hipEventSynchronize failed");
    for (int k = 0; k < HSB_TIMING_STAGES; ++k) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, h->events[kMarks * c + k], h->events[kMarks * c + k + 1]) != hipSuccess)
        return fail(h, HSB_ERR_DEVICE, "hipEventElapsedTime failed");
      acc[k] += ms;
    }
  }
  for (int k = 0; k < HSB_TIMING_STAGES; ++k) ms_avg[k] = h->n_timed ? acc[k] / h->n_timed : 0.0;
  *n_calls = h->n_timed;
  return HSB_OK;
}

int hsbuild_set_option(hsbuild_t h, int32_t option, int32_t value) {
  if (!h) return HSB_ERR_ARG;
  h->err.clear();
  switch (option) {
    case HSB_OPT_TILE_GROUP:
      if (value < 0 || value > 64) return fail(h, HSB_ERR_ARG, "tile group %d outside [0, 64]", value);
      if (value != h->tile_group) drop_graph(h);
      h->tile_group = value;
      return HSB_OK;
    case HSB_OPT_HS_WAVES:
      if (value != 4 && value != 8) return fail(h, HSB_ERR_ARG, "contraction waves must be 4 or 8 (got %d)", value);
      if (value != h->hs_waves) drop_graph(h);
      h->hs_waves = value;
      return HSB_OK;
    case HSB_OPT_SPLIT_K:
      if (value < 0 || value > 8) return fail(h, HSB_ERR_ARG, "split-K option %d outside [0, 8]", value);
      h->split_k = value;  // the batch contraction never splits: its graph stays valid
      return HSB_OK;
    default:
      return fail(h, HSB_ERR_ARG, "unknown option %d", option);
  }
}

int hsbuild_get_option(hsbuild_t h, int32_t option, int32_t* value) {
  if (!h || !value) return HSB_ERR_ARG;
  switch (option) {
    case HSB_OPT_TILE_GROUP:
      *value = h->tile_group;
      return HSB_OK;
    case HSB_OPT_HS_WAVES:
      *value = h->hs_waves;
      return HSB_OK;
    case HSB_OPT_SPLIT_K:
      *value = h->split_k;
      return HSB_OK;
    default:
      return fail(h, HSB_ERR_ARG, "unknown option %d", option);
  }
}

const char* hsbuild_last_error(hsbuild_t h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int hsbuild_host_bessel(int32_t lmax, double x, double* jl, double* djl) {
  if (lmax < 0 || lmax > HSB_MAX_LMAX || !(x >= 0.0) || !jl || !djl) return HSB_ERR_ARG;
  double j[kMaxL + 2];
  sph_bessel_seq(lmax + 1, x, j);
  sph_bessel_deriv(lmax, j, djl);
  for (int l = 0; l <= lmax; ++l) jl[l] = j[l];
  return HSB_OK;
}

int hsbuild_host_angular(int32_t lmax, const double kvec[3], double pre, void* out) {
  if (lmax < 0 || lmax > HSB_MAX_LMAX || !kvec || !out) return HSB_ERR_ARG;
  double* o = (double*)out;
  angular_visit(lmax, kvec[0], kvec[1], kvec[2], pre, [&](int L, double re, double im) {
    o[2 * L] = re;
    o[2 * L + 1] = im;
  });
  return HSB_OK;
}

int hsbuild_mfma_probe(int32_t kind, int32_t blocks, int32_t iters, void* out, size_t out_bytes, void* stream,
                       double* ops) {
  if (kind != HSB_PROBE_FP64 && kind != HSB_PROBE_INT8 && kind != HSB_PROBE_INT8_RANDOM)
    return fail(nullptr, HSB_ERR_ARG, "unknown probe kind %d", kind);
  if (blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 26) || iters % kProbeUnroll)
    return fail(nullptr, HSB_ERR_ARG, "blocks=%d or iters=%d out of range (iters: a multiple of %d)", blocks, iters,
                kProbeUnroll);
  if (!out || !ops) return fail(nullptr, HSB_ERR_ARG, "null out or ops");
  const size_t need = (size_t)blocks * 256 * (kind == HSB_PROBE_FP64 ? sizeof(double) : sizeof(unsigned));
  if (out_bytes < need) return fail(nullptr, HSB_ERR_WORKSPACE, "out holds %zu bytes, the probe writes %zu", out_bytes, need);
  // 4 waves per workgroup, 4 independent MFMA chains per wave
  *ops = (double)blocks * 4.0 * 4.0 * (double)iters * probe_ops_per_mfma(kind);
  const hipError_t e = launch_mfma_probe(kind, blocks, iters, out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(nullptr, HSB_ERR_DEVICE, "probe launch: %s", hipGetErrorString(e));
  return HSB_OK;
}

}  // extern "C"
