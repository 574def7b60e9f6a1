// Orbitals at arbitrary points from plane-wave coefficients (Sec. VI, projecting the wave
// functions).  A Bloch state stored as coefficients C_bk(G), Eq. (bloch), is evaluated at the
// points r by the direct method: per k the phase matrix P_k(r, G) = exp(i (k+G).r), common to
// every band, and the product psi_k(r, b) = sum_G P_k(r, G) C_k(G, b), here a complex FP64
// GEMM on the matrix cores (cgemm64.h) with the points as columns:
//   Y[b][r] = sum_G C[b][G] P[r][G],   psi = Y / sqrt(Omega).
// Per k: the phases are written as real and imaginary planes [points][G] and the
// coefficients repacked into planes [bands][G], both zero-padded to whole tiles and chunks,
// and one launch covers every (64-band, 128-point) tile.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "cgemm64.h"
#include "lrs_internal.h"

namespace lrs {
namespace {

// P[r][G] = exp(i (k+G).r) for r < npts, G < npw; zero in the padding.  kg [npw][3] holds k+G.
__global__ void phase_kernel(const double* kg, const double* pts, int npts, int npw, int rows,
                             int ld, double* p_re, double* p_im) {
  const long long n = (long long)rows * ld;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(i / ld), g = (int)(i - (long long)r * ld);
    double c = 0.0, s = 0.0;
    if (r < npts && g < npw) {
      const double ph = pts[3 * r] * kg[3 * g] + pts[3 * r + 1] * kg[3 * g + 1] +
                        pts[3 * r + 2] * kg[3 * g + 2];
      sincos(ph, &s, &c);
    }
    p_re[i] = c;
    p_im[i] = s;
  }
}

// coefficients of one k, complex [nb][npw] -> planes [rows][ld], zero-padded
__global__ void coef_planes_kernel(const double* coef, int nb, int npw, int rows, int ld,
                                   double* a_re, double* a_im) {
  const long long n = (long long)rows * ld;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(i / ld), g = (int)(i - (long long)b * ld);
    const bool in = b < nb && g < npw;
    const size_t o = 2 * ((size_t)b * npw + g);
    a_re[i] = in ? coef[o] : 0.0;
    a_im[i] = in ? coef[o + 1] : 0.0;
  }
}

struct ProjParams {
  const double* a_re;
  const double* a_im;   // coefficient planes [rows][ld]
  const double* p_re;
  const double* p_im;   // phase planes [prow][ld]
  int ld, nb, npts;
  double scale;         // 1 / sqrt(Omega)
  double* out;          // complex128 [nb][npts] of this k
};

// one (64-band, 128-point) tile per workgroup: blockIdx.x = point tile, blockIdx.y = band tile
__global__ __launch_bounds__(256) void project_gemm_kernel(ProjParams P) {
  __shared__ __attribute__((aligned(1024))) unsigned char slot0[CG_STAGE];
  __shared__ __attribute__((aligned(1024))) unsigned char slot1[CG_STAGE];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / CG_WN, wn = wave % CG_WN;
  const int b0 = blockIdx.y * CG_BM, r0 = blockIdx.x * CG_BN;
  const int pl = wave >> 1, hf = wave & 1, lr = lane & 15, lg = lane >> 4;
  const double* asrc[CG_AT];
#pragma unroll
  for (int t = 0; t < CG_AT; ++t)
    asrc[t] = (pl ? P.a_im : P.a_re) + (size_t)(b0 + 16 * t + lr) * P.ld + 4 * lg + 2 * hf;
  const double* bsrc[CG_BT];
#pragma unroll
  for (int t = 0; t < CG_BT; ++t)
    bsrc[t] = (pl ? P.p_im : P.p_re) + (size_t)(r0 + 16 * t + lr) * P.ld + 4 * lg + 2 * hf;
  cg_f64x4 cr[CG_MB][CG_NB], ci[CG_MB][CG_NB];
#pragma unroll
  for (int i = 0; i < CG_MB; ++i)
#pragma unroll
    for (int j = 0; j < CG_NB; ++j) {
      cr[i][j] = cg_f64x4{0, 0, 0, 0};
      ci[i][j] = cg_f64x4{0, 0, 0, 0};
    }
  cgemm64_tile(asrc, bsrc, P.ld / CG_KC, wave, lane, slot0, slot1, cr, ci);
  // element e of a lane: band 4 e + lane/16, point lane%16 of its block; 16 consecutive
  // lanes store 256 contiguous bytes
#pragma unroll
  for (int i = 0; i < CG_MB; ++i)
#pragma unroll
    for (int j = 0; j < CG_NB; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int b = b0 + (wm * CG_MB + i) * 16 + 4 * e + (lane >> 4);
        const int r = r0 + (wn * CG_NB + j) * 16 + (lane & 15);
        if (b < P.nb && r < P.npts) {
          double2* o = (double2*)P.out + (size_t)b * P.npts + r;
          *o = double2{cr[i][j][e] * P.scale, ci[i][j][e] * P.scale};
        }
      }
}

lrs_status set_err(lrs_ctx* ctx, lrs_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  ctx->err = buf;
  return st;
}

bool finite_all(const double* x, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

}  // namespace
}  // namespace lrs

using namespace lrs;

extern "C" lrs_status lrs_project_orbitals(lrs_ctx* ctx, int nk, int nb, int npw,
                                           const double* kpts_host, const double* gvec_host,
                                           const void* coef, double omega, int npts,
                                           const double* points_host, void* psi_out) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (nk <= 0 || nb <= 0 || npw <= 0 || npts <= 0)
    return set_err(ctx, LRS_EINVAL, "nk, nb, npw and npts must be positive");
  if (!kpts_host || !gvec_host || !coef || !points_host || !psi_out)
    return set_err(ctx, LRS_EINVAL, "missing argument");
  if (!(omega > 0) || !std::isfinite(omega)) return set_err(ctx, LRS_EINVAL, "omega must be positive");
  if (!finite_all(kpts_host, 3 * (size_t)nk) || !finite_all(gvec_host, 3 * (size_t)npw) ||
      !finite_all(points_host, 3 * (size_t)npts))
    return set_err(ctx, LRS_ENONFINITE, "k-points, G vectors and points must be finite");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, LRS_EDEVICE, "hipSetDevice");
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return set_err(ctx, LRS_ESTATE, "the projection allocates and synchronises; it cannot be captured");
  const int ld = (int)round_up(npw, CG_KC);
  const int rows = (int)round_up(nb, CG_BM);
  const int prow = (int)round_up(npts, CG_BN);
  const size_t bytes = (size_t)(2 * (size_t)rows * ld + 2 * (size_t)prow * ld) * 8 +
                       (size_t)(3 * (size_t)nk * npw + 3 * npts) * 8;
  // the workspace stays with the context (grown when a call needs more), so repeated calls
  // allocate nothing
  DevBuf& wb = ctx->proj_work;
  if (!wb.p || wb.bytes < bytes) {
    if (wb.p && ctx->graph_pinned)
      return set_err(ctx, LRS_ESTATE, "captured graphs read this context's buffers");
    if (wb.p) {
      (void)hipFree(wb.p);
      ctx->bytes_in_use -= wb.bytes;
      wb.p = nullptr;
      wb.bytes = 0;
    }
    if (ctx->max_bytes && ctx->bytes_in_use + bytes > ctx->max_bytes)
      return set_err(ctx, LRS_ENOMEM, "projection workspace (%zu bytes) exceeds the limit", bytes);
    if (hipMalloc(&wb.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      wb.p = nullptr;
      return set_err(ctx, LRS_ENOMEM, "projection workspace");
    }
    wb.bytes = bytes;
    ctx->bytes_in_use += bytes;
  }
  char* w = (char*)wb.p;
  double* a_re = (double*)w;
  double* a_im = a_re + (size_t)rows * ld;
  double* p_re = a_im + (size_t)rows * ld;
  double* p_im = p_re + (size_t)prow * ld;
  double* kg = p_im + (size_t)prow * ld;        // k + G for every k, [nk][npw][3]
  double* pts = kg + 3 * (size_t)nk * npw;
  hipStream_t st = ctx->stream;
  std::vector<double> kgh(3 * (size_t)nk * npw);
  for (int k = 0; k < nk; ++k)
    for (int g = 0; g < npw; ++g)
      for (int d = 0; d < 3; ++d)
        kgh[3 * ((size_t)k * npw + g) + d] = gvec_host[3 * g + d] + kpts_host[3 * k + d];
  hipError_t e = hipMemcpyAsync(pts, points_host, 3 * (size_t)npts * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(kg, kgh.data(), kgh.size() * 8, hipMemcpyHostToDevice, st);
  ProjParams P;
  P.a_re = a_re;
  P.a_im = a_im;
  P.p_re = p_re;
  P.p_im = p_im;
  P.ld = ld;
  P.nb = nb;
  P.npts = npts;
  P.scale = 1.0 / std::sqrt(omega);
  for (int k = 0; k < nk && e == hipSuccess; ++k) {
    hipLaunchKernelGGL(phase_kernel, dim3(2048), dim3(256), 0, st, kg + 3 * (size_t)k * npw, pts,
                       npts, npw, prow, ld, p_re, p_im);
    hipLaunchKernelGGL(coef_planes_kernel, dim3(2048), dim3(256), 0, st,
                       (const double*)coef + 2 * (size_t)k * nb * npw, nb, npw, rows, ld, a_re,
                       a_im);
    P.out = (double*)psi_out + 2 * (size_t)k * nb * npts;
    hipLaunchKernelGGL(project_gemm_kernel, dim3(prow / CG_BN, rows / CG_BM), dim3(256), 0, st, P);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // (the host tables are freed on return)
  if (e != hipSuccess) return set_err(ctx, LRS_EDEVICE, "projection: %s", hipGetErrorString(e));
  return LRS_OK;
}
