// Sustained matrix-core rate of the instruction mix each chi0 precision issues, on every CU
// with one wave per SIMD (the chi0 kernel's occupancy) and no memory traffic: the measured
// denominator against which the chi0 kernel's executed rate is compared, next to the
// datasheet peak.
#include <hip/hip_runtime.h>

#include "lrs_internal.h"

namespace lrs {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 b16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// Per iteration and wave, 8 (16-bit and fp8 paths) or 16 (FP32, FP64) independent accumulators
// each take: BF16X2 / FP16X2 three 32x32x16 instructions; F16F8 two 32x32x16 fp16 and one
// scaled 32x32x64 fp8 instruction (the chi0 kernel's 2 : 1 mix); FP32 and FP64 one 16x16x4
// instruction.  Flops are counted at the instruction's own rate, with an fp8 instruction
// counted as the two fp16 instructions of equal matrix-core time.
template <int PREC>
__global__ __launch_bounds__(256) void mfma_rate_kernel(long long iters, float* sink) {
  const int lane = threadIdx.x & 63;
  const float x = 1e-3f * (float)(lane + 1);
  float s = 0.f;
  if constexpr (PREC == LRS_F16F8 || PREC == LRS_FP16X2) {
    h16x8 a, b;
    i32x8 a8, b8;
    for (int e = 0; e < 8; ++e) {
      a[e] = (_Float16)x;
      b[e] = (_Float16)(x * 0.5f);
      a8[e] = 0x38383838 + lane;
      b8[e] = 0x30303030 + lane;
    }
    f32x16 acc[8];
    for (int j = 0; j < 8; ++j)
      for (int e = 0; e < 16; ++e) acc[j][e] = 0.f;
    for (long long it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[j], 0, 0, 0);
      if constexpr (PREC == LRS_F16F8) {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          acc[j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, acc[j], 0, 0, 0, 120, 0,
                                                                   109);
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(b, a, acc[j], 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, a, acc[j], 0, 0, 0);
    }
    for (int j = 0; j < 8; ++j)
      for (int e = 0; e < 16; ++e) s += acc[j][e];
  } else if constexpr (PREC == LRS_BF16X2) {
    b16x8 a, b;
    for (int e = 0; e < 8; ++e) {
      a[e] = (__bf16)x;
      b[e] = (__bf16)(x * 0.5f);
    }
    f32x16 acc[8];
    for (int j = 0; j < 8; ++j)
      for (int e = 0; e < 16; ++e) acc[j][e] = 0.f;
    for (long long it = 0; it < iters; ++it) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[j], 0, 0, 0);
    }
    for (int j = 0; j < 8; ++j)
      for (int e = 0; e < 16; ++e) s += acc[j][e];
  } else if constexpr (PREC == LRS_FP32) {
    f32x4 acc[16];
    for (int j = 0; j < 16; ++j)
      for (int e = 0; e < 4; ++e) acc[j][e] = 0.f;
    for (long long it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, 0.5f * x, acc[j], 0, 0, 0);
    }
    for (int j = 0; j < 16; ++j)
      for (int e = 0; e < 4; ++e) s += acc[j][e];
  } else {
    const double xd = x;
    f64x4 acc[16];
    for (int j = 0; j < 16; ++j)
      for (int e = 0; e < 4; ++e) acc[j][e] = 0.0;
    for (long long it = 0; it < iters; ++it) {
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xd, 0.5 * xd, acc[j], 0, 0, 0);
    }
    for (int j = 0; j < 16; ++j)
      for (int e = 0; e < 4; ++e) s += (float)acc[j][e];
  }
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// flops per wave and iteration, fp8 instructions at fp16-equivalent cost
double flops_per_iter(int prec) {
  switch (prec) {
    case LRS_F16F8: return 16.0 * 32768 + 8.0 * 65536;
    case LRS_FP16X2:
    case LRS_BF16X2: return 24.0 * 32768;
    default: return 16.0 * 2048;
  }
}

lrs_status set_err(lrs_ctx* ctx, lrs_status st, const char* msg) {
  ctx->err = msg;
  return st;
}

// the probe's small output buffer (kept in the context, within LRS_MAX_BYTES)
bool ensure_probe(lrs_ctx* ctx, size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  DevBuf& b = ctx->probe;
  if (b.p && b.bytes >= bytes) return true;
  if (b.p) {
    if (ctx->graph_pinned) return false;
    (void)hipFree(b.p);
    ctx->bytes_in_use -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  if (ctx->max_bytes && ctx->bytes_in_use + bytes > ctx->max_bytes) return false;
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return false;
  }
  b.bytes = bytes;
  ctx->bytes_in_use += bytes;
  return true;
}

}  // namespace
}  // namespace lrs

using namespace lrs;

extern "C" lrs_status lrs_mfma_rate(lrs_ctx* ctx, int prec, long long iters, double* tflops,
                                    double* ms) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (prec < LRS_FP64 || prec > LRS_F16F8) return set_err(ctx, LRS_EINVAL, "bad precision");
  if (iters <= 0 || !tflops) return set_err(ctx, LRS_EINVAL, "iters must be positive, tflops set");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, LRS_EDEVICE, "hipSetDevice");
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return set_err(ctx, LRS_ESTATE, "the rate probe synchronises; it cannot be captured");
  const int grid = ctx->num_cu;
  if (!ensure_probe(ctx, (size_t)grid * 256 * sizeof(float)))
    return set_err(ctx, LRS_ENOMEM, "rate probe output (256 floats per CU)");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return set_err(ctx, LRS_EDEVICE, "hipEventCreate");
  }
  float* sink = (float*)ctx->probe.p;
  hipError_t e = hipEventRecord(e0, ctx->stream);
  switch (prec) {
    case LRS_FP64:
      hipLaunchKernelGGL(mfma_rate_kernel<LRS_FP64>, dim3(grid), dim3(256), 0, ctx->stream, iters, sink);
      break;
    case LRS_FP32:
      hipLaunchKernelGGL(mfma_rate_kernel<LRS_FP32>, dim3(grid), dim3(256), 0, ctx->stream, iters, sink);
      break;
    case LRS_BF16X2:
      hipLaunchKernelGGL(mfma_rate_kernel<LRS_BF16X2>, dim3(grid), dim3(256), 0, ctx->stream, iters, sink);
      break;
    case LRS_FP16X2:
      hipLaunchKernelGGL(mfma_rate_kernel<LRS_FP16X2>, dim3(grid), dim3(256), 0, ctx->stream, iters, sink);
      break;
    default:
      hipLaunchKernelGGL(mfma_rate_kernel<LRS_F16F8>, dim3(grid), dim3(256), 0, ctx->stream, iters, sink);
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return set_err(ctx, LRS_EDEVICE, hipGetErrorString(e));
  const double waves = 4.0 * grid;
  *tflops = waves * (double)iters * flops_per_iter(prec) / (t * 1e-3) / 1e12;
  if (ms) *ms = t;
  return LRS_OK;
}
