// Matrix-core rate probe: every wave runs long chains of independent MFMAs on
// register operands, with no memory traffic until one store at the end.  The
// sustained rate it measures is what the contraction kernels can reach on the
// same device (FP64 16x16x4 for the complex FP64 path, int8 32x32x32 for the
// int8 split paths, on constant or on changing random operands), and, divided by
// the per-CU rate per clock, the clock the matrix cores hold under that load.
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

// 32-bit integer hash (xor-shift-multiply rounds of Wellons' "lowbias32"), for operand bytes.
__device__ __forceinline__ unsigned mix32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Four signed bytes in [-120, 120] from a hash: the spread of the residue contraction's
// operands (residues modulo m < 256, centred).
__device__ __forceinline__ int rand_bytes(unsigned key) {
  const unsigned h = mix32(key);
  unsigned r = 0u;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int v = (int)(((h >> (8 * b)) & 0xffu) % 241u) - 120;
    r |= ((unsigned)v & 0xffu) << (8 * b);
  }
  return (int)r;
}

// int8 MFMAs on operands that change every instruction: four register sets of hashed bytes,
// taken in turn, as the residue contraction feeds the matrix cores.  The matrix cores draw
// more power on such operands than on the constant bytes of k_probe_i8 and may hold a lower
// clock.  The int32 sums wrap: only the rate is of interest.
__global__ void __launch_bounds__(256) k_probe_i8_random(int iters, unsigned* __restrict__ out) {
  constexpr int kSets = 4;
  const unsigned id = blockIdx.x * 256u + threadIdx.x;
  i4v a[kSets], b[kSets];
#pragma unroll
  for (int t = 0; t < kSets; ++t)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      a[t][w] = rand_bytes(id * 64u + (unsigned)(t * 8 + w));
      b[t][w] = rand_bytes(id * 64u + (unsigned)(t * 8 + 4 + w));
    }
  i16v c[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) c[j][r] = 0;
  for (int i = 0; i < iters; i += kUnroll) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int j = 0; j < kChains; ++j)
        c[j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[(u + j) % kSets], b[(u + 2 * j + 1) % kSets], c[j], 0, 0, 0);
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
  else if (kind == 1)
    hipLaunchKernelGGL(k_probe_i8, dim3(blocks), dim3(256), 0, s, iters, (unsigned*)out);
  else
    hipLaunchKernelGGL(k_probe_i8_random, dim3(blocks), dim3(256), 0, s, iters, (unsigned*)out);
  return hipGetLastError();
}

}  // namespace hsb
