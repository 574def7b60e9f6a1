// Orbitals from plane-wave coefficients by FFT (Sec. VI, projecting the wave functions, the
// FFT route, and Eq. bloch):
//   u_bk(x_j) = sum_G C_bk(G) exp(i G.x_j)     on the grid x_j = sum_d (j_d / N_d) a_d,
//   u_bk(r)   = cubic Lagrange interpolation of u_bk(x) at the points r (cached stencils),
//   psi_bk(r) = exp(i k.r) u_bk(r) / sqrt(Omega).
// With Miller indices m (G = sum_d m_d b_d), G.x_j = 2 pi sum_d m_d j_d / N_d, so u on the grid is
// the unnormalised inverse DFT of C placed at m mod N: a zeroed box per band, the coefficients
// scattered into it, then one pass of a mixed-radix Stockham FFT along each axis, the lines of a
// pass held in LDS (16 lines per workgroup, radices 4, 2, 3, 5, sizes up to 128).  The grid
// values times the Bloch phase are the grid orbitals (lrs_set_orbitals_pw); interpolated at
// arbitrary points they are lrs_project_orbitals_fft.  Everything is FP64 and HBM-bound: each
// pass reads and writes the box once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "lrs_internal.h"

namespace lrs {
namespace {

constexpr int kMaxFFT = 128;   // longest axis (LDS: two buffers of 16 lines)
constexpr int kLines = 16;     // lines per workgroup

struct FftPlan {
  int n, nf;
  int rad[8];                  // radices in stage order
};

// n = 4^a 2^b 3^c 5^d (<= kMaxFFT), radices 4 first; false if n has another prime factor
bool make_plan(int n, FftPlan& p) {
  if (n < 1 || n > kMaxFFT) return false;
  p.n = n;
  p.nf = 0;
  int m = n;
  const int radices[4] = {4, 2, 3, 5};
  for (int r : radices) {
    while (m % r == 0 && p.nf < 8) {
      if (r == 2 && m % 4 == 0) break;     // (fours first)
      p.rad[p.nf++] = r;
      m /= r;
    }
  }
  while (m % 2 == 0 && p.nf < 8) {
    p.rad[p.nf++] = 2;
    m /= 2;
  }
  return m == 1;
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline double2 expi_turns(double t) {   // exp(2 pi i t)
  double s, c;
  sincospi(2.0 * t, &s, &c);
  return make_double2(c, s);
}

// Inverse (exp(+2 pi i ...)) Stockham stages on `nl` lines held in a[line][*]; returns the buffer
// that holds the result.  Stage with radix R after sub-transforms of size Ns: butterfly j of a
// line takes x[j + r n/R] (r < R), twiddles them by exp(2 pi i r (j mod Ns)/(Ns R)), takes their
// R-point DFT and stores it at (j / Ns) Ns R + (j mod Ns) + r Ns.
__device__ double2 (*fft_lines(double2 (*a)[kMaxFFT], double2 (*b)[kMaxFFT], const FftPlan& P,
                               int nl))[kMaxFFT] {
  int Ns = 1;
  for (int s = 0; s < P.nf; ++s) {
    const int R = P.rad[s];
    const int nbf = P.n / R;
    for (int it = threadIdx.x; it < nl * nbf; it += blockDim.x) {
      const int line = it / nbf, j = it - line * nbf;
      const int k = j % Ns;
      double2 v[5], V[5];
      for (int r = 0; r < R; ++r) {
        v[r] = a[line][j + r * nbf];
        if (r > 0 && k > 0) v[r] = cmul(v[r], expi_turns((double)(r * k) / (double)(Ns * R)));
      }
      for (int q = 0; q < R; ++q) {
        double2 acc = v[0];
        for (int r = 1; r < R; ++r) {
          const double2 w = expi_turns((double)((r * q) % R) / (double)R);
          const double2 t = cmul(v[r], w);
          acc.x += t.x;
          acc.y += t.y;
        }
        V[q] = acc;
      }
      const int d = (j / Ns) * Ns * R + k;
      for (int r = 0; r < R; ++r) b[line][d + r * Ns] = V[r];
    }
    __syncthreads();
    double2 (*t)[kMaxFFT] = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// The contiguous axis (the last): lines of P.n consecutive values, 16 per workgroup; one band
// per blockIdx.y (box stride `vol`).
__global__ void __launch_bounds__(256) fft_contig_kernel(double2* box, long long vol,
                                                         long long nlines, FftPlan P) {
  __shared__ double2 s0[kLines][kMaxFFT];
  __shared__ double2 s1[kLines][kMaxFFT];
  double2* data = box + (long long)blockIdx.y * vol;
  const long long l0 = (long long)blockIdx.x * kLines;
  const int nl = (int)min((long long)kLines, nlines - l0);
  const int n = P.n;
  for (int it = threadIdx.x; it < nl * n; it += blockDim.x) s0[it / n][it % n] = data[l0 * n + it];
  __syncthreads();
  double2 (*res)[kMaxFFT] = fft_lines(s0, s1, P, nl);
  for (int it = threadIdx.x; it < nl * n; it += blockDim.x) data[l0 * n + it] = res[it / n][it % n];
}

// A strided axis: the box as [outer][n][inner] with inner contiguous; a workgroup takes the 16
// lines (o, c0 .. c0 + 15), so that every load and store moves 16 neighbouring values.
__global__ void __launch_bounds__(256) fft_strided_kernel(double2* box, long long vol, int outer,
                                                          long long inner, FftPlan P) {
  __shared__ double2 s0[kLines][kMaxFFT];
  __shared__ double2 s1[kLines][kMaxFFT];
  double2* data = box + (long long)blockIdx.y * vol;
  const long long nblk = (inner + kLines - 1) / kLines;
  const long long o = blockIdx.x / nblk;
  const long long c0 = (blockIdx.x - o * nblk) * kLines;
  const int nl = (int)min((long long)kLines, inner - c0);
  const int n = P.n;
  const long long base = o * n * inner + c0;
  for (int it = threadIdx.x; it < kLines * n; it += blockDim.x) {
    const int i = it / kLines, c = it % kLines;
    if (c < nl) s0[c][i] = data[base + (long long)i * inner + c];
  }
  __syncthreads();
  double2 (*res)[kMaxFFT] = fft_lines(s0, s1, P, nl);
  for (int it = threadIdx.x; it < kLines * n; it += blockDim.x) {
    const int i = it / kLines, c = it % kLines;
    if (c < nl) data[base + (long long)i * inner + c] = res[c][i];
  }
}

// C_bk(G) of bands [b0, b0 + nbb) at k into the zeroed boxes: one thread per (band, G)
__global__ void scatter_kernel(const double2* coef, int nb, int npw, int b0, int nbb,
                               const int* gidx, int n0, int n1, int n2, long long vol,
                               double2* box) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nbb * npw) return;
  const int bb = (int)(t / npw), g = (int)(t - (long long)bb * npw);
  const int m0 = ((gidx[3 * g] % n0) + n0) % n0;
  const int m1 = ((gidx[3 * g + 1] % n1) + n1) % n1;
  const int m2 = ((gidx[3 * g + 2] % n2) + n2) % n2;
  box[bb * vol + ((long long)m0 * n1 + m1) * n2 + m2] = coef[(long long)(b0 + bb) * npw + g];
}

// psi at the points: 4 x 4 x 4 stencil (first nodes base[p], weights w[p][3][4]) times the Bloch
// phase; one thread per (band, point)
__global__ void interp_kernel(const double2* box, long long vol, int n0, int n1, int n2,
                              const int* base, const double* w, const double* pts, int npts,
                              double kx, double ky, double kz, double inv_sqrt_omega, int nbb,
                              double2* out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nbb * npts) return;
  const int bb = (int)(t / npts), p = (int)(t - (long long)bb * npts);
  const double2* u = box + bb * vol;
  const double* wp = w + 12 * (long long)p;
  double2 acc = make_double2(0.0, 0.0);
  for (int a = 0; a < 4; ++a) {
    const int i0 = ((base[3 * p] + a) % n0 + n0) % n0;
    for (int c = 0; c < 4; ++c) {
      const int i1 = ((base[3 * p + 1] + c) % n1 + n1) % n1;
      const double wac = wp[a] * wp[4 + c];
      const double2* row = u + ((long long)i0 * n1 + i1) * n2;
      for (int e = 0; e < 4; ++e) {
        const int i2 = ((base[3 * p + 2] + e) % n2 + n2) % n2;
        const double we = wac * wp[8 + e];
        acc.x += we * row[i2].x;
        acc.y += we * row[i2].y;
      }
    }
  }
  double s, c;
  sincos(kx * pts[3 * p] + ky * pts[3 * p + 1] + kz * pts[3 * p + 2], &s, &c);
  const double2 ph = make_double2(c * inv_sqrt_omega, s * inv_sqrt_omega);
  out[(long long)bb * npts + p] = cmul(acc, ph);
}

// grid orbitals: the box values times exp(i k.x_j) / sqrt(Omega), x_j = sum_d (j_d / N_d) a_d;
// one thread per (band, grid point), output in the box's own order
__global__ void grid_out_kernel(const double2* box, long long vol, int n0, int n1, int n2,
                                const double* cell, double kx, double ky, double kz,
                                double inv_sqrt_omega, int nbb, double2* out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nbb * vol) return;
  const long long bb = t / vol, idx = t - bb * vol;
  const int j2 = (int)(idx % n2), j1 = (int)((idx / n2) % n1), j0 = (int)(idx / ((long long)n1 * n2));
  const double f0 = (double)j0 / n0, f1 = (double)j1 / n1, f2 = (double)j2 / n2;
  const double x = f0 * cell[0] + f1 * cell[3] + f2 * cell[6];
  const double y = f0 * cell[1] + f1 * cell[4] + f2 * cell[7];
  const double z = f0 * cell[2] + f1 * cell[5] + f2 * cell[8];
  double s, c;
  sincos(kx * x + ky * y + kz * z, &s, &c);
  out[t] = cmul(box[t], make_double2(c * inv_sqrt_omega, s * inv_sqrt_omega));
}

lrs_status set_err(lrs_ctx* ctx, lrs_status st, const char* msg) {
  ctx->err = msg;
  return st;
}

hipError_t ensure_fft(lrs_ctx* ctx, DevBuf& b, size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  if (b.p && b.bytes >= bytes) return hipSuccess;
  if (b.p) {
    if (ctx->graph_pinned) return hipErrorIllegalState;
    (void)hipFree(b.p);
    ctx->bytes_in_use -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  if (ctx->max_bytes && ctx->bytes_in_use + bytes > ctx->max_bytes) return hipErrorOutOfMemory;
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return hipErrorOutOfMemory;
  }
  b.bytes = bytes;
  ctx->bytes_in_use += bytes;
  return hipSuccess;
}

// Shared driver: u on the N0 x N1 x N2 grid per (k, band batch), then either interpolation to
// `npts` points (psi_pts [nk][nb][npts]) or the grid orbitals (psi_grid [nk][nb][vol]).
lrs_status fft_route(lrs_ctx* ctx, int nk, int nb, int npw, const double* kpts,
                     const double* cell, const int* gidx, const double2* coef, double omega,
                     const int* nfft, int npts, const double* points, double2* psi_pts,
                     double2* psi_grid) {
  FftPlan plan[3];
  for (int d = 0; d < 3; ++d)
    if (!make_plan(nfft[d], plan[d]))
      return set_err(ctx, LRS_EUNSUPPORTED, "each FFT size must be 2^a 3^b 5^c and at most 128");
  for (int g = 0; g < npw; ++g)
    for (int d = 0; d < 3; ++d)
      if (2 * std::abs(gidx[3 * g + d]) >= nfft[d])
        return set_err(ctx, LRS_EINVAL, "the FFT grid must hold every plane wave: N_d > 2 |m_d|");
  const int n0 = nfft[0], n1 = nfft[1], n2 = nfft[2];
  const long long vol = (long long)n0 * n1 * n2;
  // interpolation stencils, once for all bands and k: first node and the cubic weights of the
  // nodes at offsets -1, 0, 1, 2 from floor(grid coordinate)
  std::vector<int> base;
  std::vector<double> wts;
  if (psi_pts) {
    const double* a = cell;
    const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                       a[2] * (a[3] * a[7] - a[4] * a[6]);
    double ai[9];   // A^-1 (rows of A are the lattice vectors); fractional f = r A^-1
    ai[0] = (a[4] * a[8] - a[5] * a[7]) / det;
    ai[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    ai[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    ai[3] = (a[5] * a[6] - a[3] * a[8]) / det;
    ai[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    ai[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    ai[6] = (a[3] * a[7] - a[4] * a[6]) / det;
    ai[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    ai[8] = (a[0] * a[4] - a[1] * a[3]) / det;
    base.resize((size_t)3 * npts);
    wts.resize((size_t)12 * npts);
    const double nodes[4] = {-1.0, 0.0, 1.0, 2.0};
    for (int p = 0; p < npts; ++p) {
      const double* r = points + 3 * (size_t)p;
      for (int d = 0; d < 3; ++d) {
        const double f = r[0] * ai[d] + r[1] * ai[3 + d] + r[2] * ai[6 + d];
        const double g = f * nfft[d];
        const double fl = std::floor(g);
        const double t = g - fl;
        base[3 * (size_t)p + d] = (int)fl - 1;
        for (int q = 0; q < 4; ++q) {
          double v = 1.0;
          for (int s = 0; s < 4; ++s)
            if (s != q) v *= (t - nodes[s]) / (nodes[q] - nodes[s]);
          wts[12 * (size_t)p + 4 * d + q] = v;
        }
      }
    }
  }
  // workspace: gidx | cell | stencils | points | boxes of a band batch (at most 1 GiB)
  const size_t b_small = 256 + (size_t)npw * 12 + 9 * 8 + (size_t)npts * (12 + 96 + 24) + 1024;
  const int nbb = (int)std::max<long long>(1, std::min<long long>(nb, (1LL << 30) / (vol * 16)));
  hipError_t e = ensure_fft(ctx, ctx->fft_work, b_small + (size_t)nbb * vol * 16 + 256);
  if (e == hipErrorIllegalState)
    return set_err(ctx, LRS_ESTATE, "captured graphs read this context's buffers");
  if (e != hipSuccess) return set_err(ctx, LRS_ENOMEM, "FFT workspace");
  unsigned char* w = (unsigned char*)ctx->fft_work.p;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = w + off;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  int* d_gidx = (int*)take((size_t)npw * 12);
  double* d_cell = (double*)take(72);
  int* d_base = (int*)take((size_t)npts * 12 + 1);
  double* d_w = (double*)take((size_t)npts * 96 + 1);
  double* d_pts = (double*)take((size_t)npts * 24 + 1);
  double2* box = (double2*)take((size_t)nbb * vol * 16);
  hipStream_t st = ctx->stream;
  e = hipMemcpyAsync(d_gidx, gidx, (size_t)npw * 12, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_cell, cell, 72, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && psi_pts) {
    e = hipMemcpyAsync(d_base, base.data(), (size_t)npts * 12, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_w, wts.data(), (size_t)npts * 96, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_pts, points, (size_t)npts * 24, hipMemcpyHostToDevice, st);
  }
  const double iso = 1.0 / std::sqrt(omega);
  for (int k = 0; k < nk && e == hipSuccess; ++k) {
    const double* kv = kpts + 3 * k;
    for (int b0 = 0; b0 < nb && e == hipSuccess; b0 += nbb) {
      const int nbt = std::min(nbb, nb - b0);
      e = launch_fill_zero(box, (size_t)nbt * vol * 16, st);
      if (e != hipSuccess) break;
      const long long ns = (long long)nbt * npw;
      hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st,
                         coef + (size_t)k * nb * npw, nb, npw, b0, nbt, d_gidx, n0, n1, n2, vol,
                         box);
      // last axis (contiguous lines), then the middle axis, then the first
      hipLaunchKernelGGL(fft_contig_kernel, dim3((unsigned)((vol / n2 + kLines - 1) / kLines), nbt),
                         dim3(256), 0, st, box, vol, vol / n2, plan[2]);
      const long long nb1 = (n2 + kLines - 1) / kLines;
      hipLaunchKernelGGL(fft_strided_kernel, dim3((unsigned)(n0 * nb1), nbt), dim3(256), 0, st,
                         box, vol, n0, (long long)n2, plan[1]);
      const long long inner0 = (long long)n1 * n2;
      hipLaunchKernelGGL(fft_strided_kernel,
                         dim3((unsigned)((inner0 + kLines - 1) / kLines), nbt), dim3(256), 0, st,
                         box, vol, 1, inner0, plan[0]);
      if (psi_pts) {
        const long long nt = (long long)nbt * npts;
        hipLaunchKernelGGL(interp_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st,
                           box, vol, n0, n1, n2, d_base, d_w, d_pts, npts, kv[0], kv[1], kv[2],
                           iso, nbt, psi_pts + ((size_t)k * nb + b0) * npts);
      } else {
        const long long nt = (long long)nbt * vol;
        hipLaunchKernelGGL(grid_out_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st,
                           box, vol, n0, n1, n2, d_cell, kv[0], kv[1], kv[2], iso, nbt,
                           psi_grid + ((size_t)k * nb + b0) * vol);
      }
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // host tables are freed on return
  if (e != hipSuccess) {
    ctx->err = std::string("FFT projection: ") + hipGetErrorString(e);
    return LRS_EDEVICE;
  }
  return LRS_OK;
}

// shared host-side validation of the plane-wave inputs
lrs_status check_pw(lrs_ctx* ctx, int nk, int nb, int npw, const double* kpts,
                    const double* cell, const int* gidx, const void* coef, double omega,
                    const int* nfft) {
  if (nk < 1 || nb < 1 || npw < 1 || !kpts || !cell || !gidx || !coef || !nfft || !(omega > 0))
    return set_err(ctx, LRS_EINVAL, "need nk, nb, npw >= 1, omega > 0 and every array");
  for (int i = 0; i < 3 * nk; ++i)
    if (!std::isfinite(kpts[i])) return set_err(ctx, LRS_ENONFINITE, "non-finite k-point");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(cell[i])) return set_err(ctx, LRS_ENONFINITE, "non-finite lattice vector");
  const double* a = cell;
  const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                     a[2] * (a[3] * a[7] - a[4] * a[6]);
  if (!(std::fabs(det) > 0)) return set_err(ctx, LRS_EINVAL, "singular lattice");
  if (std::fabs(std::fabs(det) - omega) > 1e-9 * omega)
    return set_err(ctx, LRS_EINVAL, "omega must be the volume of the cell");
  return LRS_OK;
}

}  // namespace
}  // namespace lrs

using namespace lrs;

extern "C" lrs_status lrs_project_orbitals_fft(lrs_ctx* ctx, int nk, int nb, int npw,
                                               const double* kpts_host, const double* cell_host,
                                               const int* gidx_host, const void* coef,
                                               double omega, const int* nfft_host, int npts,
                                               const double* points_host, void* psi_out) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  lrs_status s = check_pw(ctx, nk, nb, npw, kpts_host, cell_host, gidx_host, coef, omega, nfft_host);
  if (s != LRS_OK) return s;
  if (npts < 1 || !points_host || !psi_out) return set_err(ctx, LRS_EINVAL, "need points and psi_out");
  for (long long i = 0; i < 3LL * npts; ++i)
    if (!std::isfinite(points_host[i])) return set_err(ctx, LRS_ENONFINITE, "non-finite point");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, LRS_EDEVICE, "device");
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess) return set_err(ctx, LRS_EDEVICE, "device");
  if (cs != hipStreamCaptureStatusNone)
    return set_err(ctx, LRS_ESTATE, "the FFT projection copies host tables; it cannot be captured");
  return fft_route(ctx, nk, nb, npw, kpts_host, cell_host, gidx_host, (const double2*)coef, omega,
                   nfft_host, npts, points_host, (double2*)psi_out, nullptr);
}

extern "C" lrs_status lrs_set_orbitals_pw(lrs_ctx* ctx, int nk, int nb, int nocc, int spin_factor,
                                          const double* energies_host, double mu, double delta,
                                          const double* kpts_host, const double* cell_host,
                                          const int* gidx_host, const void* coef, int npw,
                                          double omega, const int* ngrid_host) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  lrs_status s = check_pw(ctx, nk, nb, npw, kpts_host, cell_host, gidx_host, coef, omega, ngrid_host);
  if (s != LRS_OK) return s;
  s = lrs_check_bands(nk, nb, nocc, energies_host, mu, delta);
  if (s != LRS_OK) return set_err(ctx, s, "invalid band set (see lrs_check_bands)");
  if (ctx->graph_pinned)
    return set_err(ctx, LRS_ESTATE, "captured graphs read this context's buffers; call "
                   "lrs_release_graphs once those graphs are gone");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, LRS_EDEVICE, "device");
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess) return set_err(ctx, LRS_EDEVICE, "device");
  if (cs != hipStreamCaptureStatusNone)
    return set_err(ctx, LRS_ESTATE, "lrs_set_orbitals_pw allocates; it cannot be captured");
  const long long vol = (long long)ngrid_host[0] * ngrid_host[1] * ngrid_host[2];
  if (vol > (1LL << 28)) return set_err(ctx, LRS_EINVAL, "grid too large");
  // the grid orbitals, then the ordinary packing of lrs_set_orbitals
  const size_t bytes = (size_t)nk * nb * vol * 16;
  if (ctx->max_bytes && ctx->bytes_in_use + bytes > ctx->max_bytes)
    return set_err(ctx, LRS_ENOMEM, "grid orbitals would exceed LRS_MAX_BYTES");
  void* grid = nullptr;
  if (hipMalloc(&grid, bytes) != hipSuccess || !grid) {
    (void)hipGetLastError();
    return set_err(ctx, LRS_ENOMEM, "grid orbitals");
  }
  ctx->bytes_in_use += bytes;
  s = fft_route(ctx, nk, nb, npw, kpts_host, cell_host, gidx_host, (const double2*)coef, omega,
                ngrid_host, 0, nullptr, nullptr, (double2*)grid);
  if (s == LRS_OK)
    s = lrs_set_orbitals(ctx, nk, nb, nocc, spin_factor, energies_host, mu, delta, grid, (int)vol,
                         omega / (double)vol);
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipFree(grid);
  ctx->bytes_in_use -= bytes;
  return s;
}
