// Matrix-core rate probe: every wave runs long chains of independent MFMAs on
// register operands, with no memory traffic until one store at the end.  The
// sustained rate it measures is what the contraction kernels can reach on the
// same device (FP64 16x16x4 for the complex FP64 path, int8 32x32x32 for the
// int8 split path), and, divided by the per-CU rate per clock, the clock the
// matrix cores hold under that load.
#include "hs_internal.h"

namespace hsb {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));

constexpr int kChains = 4;  // independent accumulators per wave
constexpr int kUnroll = kProbeUnroll;

__global__ void __launch_bounds__(256) k_probe_f64(int iters, double* __restrict__ out) {
  const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * blockIdx.x;
  d4 c[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) c[j] = d4{0.0, 0.0, 0.0, 0.0};
  // kUnroll MFMAs per chain between loop back edges, where the compiler may copy
  // the accumulators between register files
  for (int i = 0; i < iters; i += kUnroll) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int j = 0; j < kChains; ++j) c[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[j], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_probe_i8(int iters, unsigned* __restrict__ out) {
  // bytes of 0 or 1: every product is 0 or 1, so no sum nears the int32 range
  const i4v a = i4v{0x01010101, (int)(threadIdx.x & 1), 0x00010001, 0x01000100};
  const i4v b = i4v{0x01010101, 0x01000001, (int)(blockIdx.x & 1), 0x00000101};
  i16v c[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) c[j][r] = 0;
  for (int i = 0; i < iters; i += kUnroll) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int j = 0; j < kChains; ++j) c[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c[j], 0, 0, 0);
  }
  unsigned s = 0u;
#pragma unroll
  for (int j = 0; j < kChains; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += (unsigned)c[j][r];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

double probe_ops_per_mfma(int kind) { return kind == 0 ? 2.0 * 16 * 16 * 4 : 2.0 * 32 * 32 * 32; }

hipError_t launch_mfma_probe(int kind, int blocks, int iters, void* out, hipStream_t s) {
  if (kind == 0)
    hipLaunchKernelGGL(k_probe_f64, dim3(blocks), dim3(256), 0, s, iters, (double*)out);
  else
    hipLaunchKernelGGL(k_probe_i8, dim3(blocks), dim3(256), 0, s, iters, (unsigned*)out);
  return hipGetLastError();
}

}  // namespace hsb
