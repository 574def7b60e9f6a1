// Orbitals from plane-wave coefficients by FFT (Sec. VI, projecting the wave functions, the
// FFT route, and Eq. bloch):
//   u_bk(x_j) = sum_G C_bk(G) exp(i G.x_j)     on the grid x_j = sum_d (j_d / N_d) a_d,
//   u_bk(r)   = cubic Lagrange interpolation of u_bk(x) at the points r (cached stencils),
//   psi_bk(r) = exp(i k.r) u_bk(r) / sqrt(Omega).
// With Miller indices m (G = sum_d m_d b_d), G.x_j = 2 pi sum_d m_d j_d / N_d, so u on the grid is
// the unnormalised inverse DFT of C placed at m mod N: the coefficients scattered into a box per
// band, then one pass of a mixed-radix Stockham FFT along each axis, the lines of a pass held in
// LDS (16 lines per workgroup, radices 4, 2, 3, 5, sizes up to 128, roots from a table).  The
// coefficients fill only the sub-box S_0 x S_1 x S_2 of the indices m mod N with |m_d| <= M_d
// (S_d = {0..M_d} and {N_d - M_d..N_d - 1}), so the passes are pruned: axis 2 runs on the lines
// of S_0 x S_1 only, axis 1 on the slabs of S_0 only, axis 0 on every line, and each pass reads
// only the support of its axis (the rest of a line is zero), so nothing but the sub-box is
// cleared.  The grid values times the Bloch phase are the grid orbitals
// (lrs_set_orbitals_pw); interpolated at arbitrary points they are lrs_project_orbitals_fft.
// Everything is FP64 and HBM-bound: with four-fold oversampling the passes move about 1.6 box
// volumes per band instead of 6.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "lrs_internal.h"

namespace lrs {
namespace {

constexpr int kMaxFFT = 128;   // longest axis (LDS: two buffers of 16 lines, 66 KiB at most)
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

// The support {0..m} and {n - m..n - 1} of an axis (m < 0: the whole axis): its a-th index,
// its size, and whether index i lies in it.
__host__ __device__ inline int sup_at(int a, int m, int n) {
  return (m < 0 || a <= m) ? a : a + n - 2 * m - 1;
}
__host__ __device__ inline int sup_count(int m, int n) { return m < 0 ? n : 2 * m + 1; }
__device__ inline bool in_sup(int i, int m, int n) { return m < 0 || i <= m || i >= n - m; }

// tw[m] = exp(2 pi i m / n), m < n: every root a stage needs is one of these (its order Ns R
// divides n), so a workgroup fills the table once instead of evaluating sines per butterfly
__device__ inline void fill_twiddles(double2* tw, int n) {
  for (int m = threadIdx.x; m < n; m += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)m / (double)n, &s, &c);
    tw[m] = make_double2(c, s);
  }
}

// Inverse (exp(+2 pi i ...)) Stockham stages on `nl` lines held in a[line * ld + *] (ld = n | 1:
// an odd stride, so that the 16 lines' values at one index fall in different LDS banks); returns
// the buffer that holds the result.  Stage with radix R after sub-transforms of size Ns: butterfly j of a
// line takes x[j + r n/R] (r < R), twiddles them by exp(2 pi i r (j mod Ns)/(Ns R)), takes their
// R-point DFT and stores it at (j / Ns) Ns R + (j mod Ns) + r Ns.  Roots come from tw.
__device__ double2* fft_lines(double2* a, double2* b, const double2* tw, const FftPlan& P,
                              int nl, int ld) {
  int Ns = 1;
  const int n = P.n;
  for (int s = 0; s < P.nf; ++s) {
    const int R = P.rad[s];
    const int nbf = n / R;
    const int tstep = n / (Ns * R);     // exp(2 pi i r k / (Ns R)) = tw[r k tstep]
    for (int it = threadIdx.x; it < nl * nbf; it += blockDim.x) {
      const int line = it / nbf, j = it - line * nbf;
      const int k = j % Ns;
      double2 v[5], V[5];
      for (int r = 0; r < R; ++r) {
        v[r] = a[line * ld + j + r * nbf];
        if (r > 0 && k > 0) v[r] = cmul(v[r], tw[r * k * tstep]);
      }
      for (int q = 0; q < R; ++q) {
        double2 acc = v[0];
        for (int r = 1; r < R; ++r) {
          const double2 t = cmul(v[r], tw[((r * q) % R) * nbf]);
          acc.x += t.x;
          acc.y += t.y;
        }
        V[q] = acc;
      }
      const int d = (j / Ns) * Ns * R + k;
      for (int r = 0; r < R; ++r) b[line * ld + d + r * Ns] = V[r];
    }
    __syncthreads();
    double2* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// The contiguous axis (the last): the lines (i0, i1) of S_0 x S_1 (supports m0, m1 of axes of
// n0, n1), P.n consecutive values each, 16 per workgroup, reading the support m2 of the line
// only; one band per blockIdx.y (box stride `vol`).
__global__ void __launch_bounds__(256) fft_contig_kernel(double2* box, long long vol, int m0,
                                                         int n0, int m1, int n1, int m2,
                                                         FftPlan P) {
  // dynamic LDS: two buffers of kLines lines of P.n values, then the twiddle table
  extern __shared__ double2 smem[];
  __shared__ long long start[kLines];
  double2* data = box + (long long)blockIdx.y * vol;
  const int c1 = sup_count(m1, n1);
  const long long nlines = (long long)sup_count(m0, n0) * c1;
  const long long l0 = (long long)blockIdx.x * kLines;
  const int nl = (int)min((long long)kLines, nlines - l0);
  const int n = P.n, ld = n | 1;
  double2* s0 = smem;
  double2* s1 = smem + kLines * ld;
  double2* tw = smem + 2 * kLines * ld;
  if (threadIdx.x < nl) {
    const long long l = l0 + threadIdx.x;
    const int i0 = sup_at((int)(l / c1), m0, n0), i1 = sup_at((int)(l % c1), m1, n1);
    start[threadIdx.x] = ((long long)i0 * n1 + i1) * n;
  }
  fill_twiddles(tw, n);
  __syncthreads();
  for (int it = threadIdx.x; it < nl * n; it += blockDim.x) {
    const int line = it / n, i = it % n;
    s0[line * ld + i] = in_sup(i, m2, n) ? data[start[line] + i] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const double2* res = fft_lines(s0, s1, tw, P, nl, ld);
  for (int it = threadIdx.x; it < nl * n; it += blockDim.x)
    data[start[it / n] + it % n] = res[(it / n) * ld + it % n];
}

// A strided axis: the box as [outer][n][inner] with inner contiguous, outer restricted to the
// support mo of an axis of no values; a workgroup takes the 16 lines (o, c0 .. c0 + 15), so that
// every load and store moves 16 neighbouring values, and reads the support ml of its axis only.
__global__ void __launch_bounds__(256) fft_strided_kernel(double2* box, long long vol, int mo,
                                                          int no, long long inner, int ml,
                                                          FftPlan P) {
  extern __shared__ double2 smem[];   // as in fft_contig_kernel
  double2* data = box + (long long)blockIdx.y * vol;
  const long long nblk = (inner + kLines - 1) / kLines;
  const long long o = sup_at((int)(blockIdx.x / nblk), mo, no);
  const long long c0 = (blockIdx.x % nblk) * kLines;
  const int nl = (int)min((long long)kLines, inner - c0);
  const int n = P.n;
  const long long base = o * n * inner + c0;
  const int ld = n | 1;
  double2* s0 = smem;
  double2* s1 = smem + kLines * ld;
  double2* tw = smem + 2 * kLines * ld;
  fill_twiddles(tw, n);
  for (int it = threadIdx.x; it < kLines * n; it += blockDim.x) {
    const int i = it / kLines, c = it % kLines;
    if (c < nl)
      s0[c * ld + i] =
          in_sup(i, ml, n) ? data[base + (long long)i * inner + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const double2* res = fft_lines(s0, s1, tw, P, nl, ld);
  for (int it = threadIdx.x; it < kLines * n; it += blockDim.x) {
    const int i = it / kLines, c = it % kLines;
    if (c < nl) data[base + (long long)i * inner + c] = res[c * ld + i];
  }
}

// An axis as a direct sum over its support: the box as [outer][n][inner] (outer restricted to
// the support mo of an axis of no values), each output j of a column (o, c) is the sum over the
// c_l <= kMaxSup indices m of the axis's support ml of u(m) exp(2 pi i m j / n).  One thread
// per (band, o, c): it reads its c_l values (a wave reads 64 neighbouring columns of a row) and
// writes all n outputs the same way, so the pass streams the box in long runs; the root index
// m j mod n is the same across the workgroup, so the table read is a broadcast.  Where the
// support is short (four-fold oversampling: a quarter of the axis) this costs fewer memory
// passes than staging lines through LDS, and the arithmetic stays far below the memory time.
constexpr int kMaxSup = 32;
__global__ void __launch_bounds__(256) axis_dft_kernel(double2* box, long long vol, int mo,
                                                       int no, int n, long long inner, int ml,
                                                       int nbb) {
  __shared__ double2 tw[kMaxFFT];
  fill_twiddles(tw, n);
  __syncthreads();
  const long long per = (long long)sup_count(mo, no) * inner;   // columns per band
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nbb * per) return;
  const long long r = t % per;
  const long long o = sup_at((int)(r / inner), mo, no);
  double2* u = box + (t / per) * vol + o * n * inner + r % inner;
  const int cl = sup_count(ml, n);
  double2 x[kMaxSup];
  int m[kMaxSup], idx[kMaxSup];
#pragma unroll
  for (int a = 0; a < kMaxSup; ++a) {
    m[a] = a < cl ? sup_at(a, ml, n) : 0;
    x[a] = a < cl ? u[(long long)m[a] * inner] : make_double2(0.0, 0.0);
    idx[a] = 0;
  }
  for (int j = 0; j < n; ++j) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < kMaxSup; ++a) {
      if (a < cl) {
        const double2 w = tw[idx[a]];
        acc.x += x[a].x * w.x - x[a].y * w.y;
        acc.y += x[a].x * w.y + x[a].y * w.x;
        idx[a] += m[a];
        idx[a] -= idx[a] >= n ? n : 0;
      }
    }
    u[(long long)j * inner] = acc;
  }
}

// clears the sub-box S_0 x S_1 x S_2 of nbb boxes; one thread per value
__global__ void zero_sub_kernel(double2* box, long long vol, int m0, int n0, int m1, int n1,
                                int m2, int n2, int nbb) {
  const int c0 = sup_count(m0, n0), c1 = sup_count(m1, n1), c2 = sup_count(m2, n2);
  const long long per = (long long)c0 * c1 * c2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= per * nbb) return;
  const long long bb = t / per, r = t - bb * per;
  const int a2 = (int)(r % c2), a1 = (int)((r / c2) % c1), a0 = (int)(r / ((long long)c1 * c2));
  box[bb * vol + ((long long)sup_at(a0, m0, n0) * n1 + sup_at(a1, m1, n1)) * n2 +
      sup_at(a2, m2, n2)] = make_double2(0.0, 0.0);
}

// exp(i k.r) / sqrt(Omega) at each point (the Bloch phase of the interpolated values)
__global__ void point_phase_kernel(const double* pts, int npts, double kx, double ky, double kz,
                                   double inv_sqrt_omega, double2* ph) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  double s, c;
  sincos(kx * pts[3 * p] + ky * pts[3 * p + 1] + kz * pts[3 * p + 2], &s, &c);
  ph[p] = make_double2(c * inv_sqrt_omega, s * inv_sqrt_omega);
}

// exp(i k.(j / N_d) a_d) per axis d and index j (tables of n0, n1, n2 values one after the
// other); their product over the axes, over sqrt(Omega), is the grid point's Bloch phase
__global__ void axis_phase_kernel(const double* cell, double kx, double ky, double kz, int n0,
                                  int n1, int n2, double2* ph) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n0 + n1 + n2) return;
  const int d = t < n0 ? 0 : (t < n0 + n1 ? 1 : 2);
  const int j = t - (d == 0 ? 0 : (d == 1 ? n0 : n0 + n1));
  const int nd = d == 0 ? n0 : (d == 1 ? n1 : n2);
  const double f = (double)j / nd;
  double s, c;
  sincos(f * (kx * cell[3 * d] + ky * cell[3 * d + 1] + kz * cell[3 * d + 2]), &s, &c);
  ph[t] = make_double2(c, s);
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

// psi at the points: 4 x 4 x 4 stencil (first nodes base[p] in [0, n), weights w[p][3][4]) times
// the Bloch phase ph[p]; one thread per (band, point).  The points come sorted by their first
// node (neighbouring threads gather neighbouring grid values); order[p] is the caller's index.
__global__ void interp_kernel(const double2* box, long long vol, int n0, int n1, int n2,
                              const int* base, const double* w, const double2* ph,
                              const int* order, int npts, int nbb, double2* out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nbb * npts) return;
  const int bb = (int)(t / npts), p = (int)(t - (long long)bb * npts);
  const double2* u = box + bb * vol;
  const double* wp = w + 12 * (long long)p;
  // the four node indices per axis, wrapped into the box (first nodes lie in [0, n), so
  // three subtractions cover any n >= 1)
  auto wrap = [](int x, int n) {
    x -= x >= n ? n : 0;
    x -= x >= n ? n : 0;
    return x - (x >= n ? n : 0);
  };
  int i0[4], i1[4], i2[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    i0[a] = wrap(base[3 * p] + a, n0);
    i1[a] = wrap(base[3 * p + 1] + a, n1);
    i2[a] = wrap(base[3 * p + 2] + a, n2);
  }
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double wac = wp[a] * wp[4 + c];
      const double2* row = u + ((long long)i0[a] * n1 + i1[c]) * n2;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double we = wac * wp[8 + e];
        const double2 v = row[i2[e]];
        acc.x += we * v.x;
        acc.y += we * v.y;
      }
    }
  }
  out[(long long)bb * npts + order[p]] = cmul(acc, ph[p]);
}

// grid orbitals: the box values times exp(i k.x_j) / sqrt(Omega), x_j = sum_d (j_d / N_d) a_d;
// one thread per (band, grid point), output in the box's own order
__global__ void grid_out_kernel(const double2* box, long long vol, int n0, int n1, int n2,
                                const double2* aph, double inv_sqrt_omega, int nbb,
                                double2* out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nbb * vol) return;
  const long long idx = t % vol;
  const int j2 = (int)(idx % n2), j1 = (int)((idx / n2) % n1), j0 = (int)(idx / ((long long)n1 * n2));
  double2 ph = cmul(cmul(aph[j0], aph[n0 + j1]), aph[n0 + n1 + j2]);
  ph.x *= inv_sqrt_omega;
  ph.y *= inv_sqrt_omega;
  out[t] = cmul(box[t], ph);
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
  // the coefficients' support per axis: |m_d| <= M_d (2 M_d + 1 <= N_d, checked above)
  int M[3] = {0, 0, 0};
  for (int g = 0; g < npw; ++g)
    for (int d = 0; d < 3; ++d) M[d] = std::max(M[d], std::abs(gidx[3 * g + d]));
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
        // first node, reduced into [0, N_d) (the grid is periodic)
        const long long b = ((long long)fl - 1) % nfft[d];
        base[3 * (size_t)p + d] = (int)(b < 0 ? b + nfft[d] : b);
        for (int q = 0; q < 4; ++q) {
          double v = 1.0;
          for (int s = 0; s < 4; ++s)
            if (s != q) v *= (t - nodes[s]) / (nodes[q] - nodes[s]);
          wts[12 * (size_t)p + 4 * d + q] = v;
        }
      }
    }
  }
  // points in the order of their first node (lexicographic), stencils and coordinates with them
  std::vector<int> order, base_s;
  std::vector<double> wts_s, pts_s;
  if (psi_pts) {
    order.resize(npts);
    for (int p = 0; p < npts; ++p) order[p] = p;
    std::sort(order.begin(), order.end(), [&](int x, int y) {
      for (int d = 0; d < 3; ++d)
        if (base[3 * (size_t)x + d] != base[3 * (size_t)y + d])
          return base[3 * (size_t)x + d] < base[3 * (size_t)y + d];
      return x < y;
    });
    base_s.resize(base.size());
    wts_s.resize(wts.size());
    pts_s.resize((size_t)3 * npts);
    for (int q = 0; q < npts; ++q) {
      const size_t p = order[q];
      for (int d = 0; d < 3; ++d) {
        base_s[3 * (size_t)q + d] = base[3 * p + d];
        pts_s[3 * (size_t)q + d] = points[3 * p + d];
      }
      for (int i = 0; i < 12; ++i) wts_s[12 * (size_t)q + i] = wts[12 * p + i];
    }
  }
  // workspace: gidx | cell | stencils | points | phases | boxes of a band batch (at most 1 GiB)
  const size_t b_small = 256 + (size_t)npw * 12 + 9 * 8 + (size_t)npts * (12 + 96 + 24 + 16 + 4) +
                         (size_t)(n0 + n1 + n2) * 16 + 1792;
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
  int* d_order = (int*)take((size_t)npts * 4 + 1);
  double2* d_ph = (double2*)take((size_t)std::max(npts, n0 + n1 + n2) * 16);
  double2* box = (double2*)take((size_t)nbb * vol * 16);
  hipStream_t st = ctx->stream;
  e = hipMemcpyAsync(d_gidx, gidx, (size_t)npw * 12, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_cell, cell, 72, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && psi_pts) {
    e = hipMemcpyAsync(d_base, base_s.data(), (size_t)npts * 12, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_w, wts_s.data(), (size_t)npts * 96, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_pts, pts_s.data(), (size_t)npts * 24, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_order, order.data(), (size_t)npts * 4, hipMemcpyHostToDevice, st);
  }
  const double iso = 1.0 / std::sqrt(omega);
  const int c0 = sup_count(M[0], n0), c1 = sup_count(M[1], n1), c2 = sup_count(M[2], n2);
  // two line buffers and the twiddle table of a pass along an axis of n values
  auto lds_bytes = [](int n) {
    return (unsigned)((2 * kLines * (n | 1) + n) * sizeof(double2));
  };
  {
    // (above 64 KiB of dynamic LDS, that is for axes longer than 123, a kernel must ask)
    const int most = (int)lds_bytes(kMaxFFT);
    hipError_t ea = hipFuncSetAttribute((const void*)fft_contig_kernel,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, most);
    if (ea == hipSuccess)
      ea = hipFuncSetAttribute((const void*)fft_strided_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, most);
    if (ea != hipSuccess) {
      ctx->err = std::string("FFT projection: ") + hipGetErrorString(ea);
      return LRS_EDEVICE;
    }
  }
  for (int k = 0; k < nk && e == hipSuccess; ++k) {
    const double* kv = kpts + 3 * k;
    if (psi_pts)
      hipLaunchKernelGGL(point_phase_kernel, dim3((npts + 255) / 256), dim3(256), 0, st, d_pts,
                         npts, kv[0], kv[1], kv[2], iso, d_ph);
    else
      hipLaunchKernelGGL(axis_phase_kernel, dim3((n0 + n1 + n2 + 255) / 256), dim3(256), 0, st,
                         d_cell, kv[0], kv[1], kv[2], n0, n1, n2, d_ph);
    for (int b0 = 0; b0 < nb && e == hipSuccess; b0 += nbb) {
      const int nbt = std::min(nbb, nb - b0);
      const long long nz = (long long)c0 * c1 * c2 * nbt;
      hipLaunchKernelGGL(zero_sub_kernel, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, st,
                         box, vol, M[0], n0, M[1], n1, M[2], n2, nbt);
      const long long ns = (long long)nbt * npw;
      hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st,
                         coef + (size_t)k * nb * npw, nb, npw, b0, nbt, d_gidx, n0, n1, n2, vol,
                         box);
      // last axis on the lines of S_0 x S_1, the middle axis on the slabs of S_0, the first
      // axis everywhere
      const long long l2 = (long long)c0 * c1;
      hipLaunchKernelGGL(fft_contig_kernel, dim3((unsigned)((l2 + kLines - 1) / kLines), nbt),
                         dim3(256), lds_bytes(n2), st, box, vol, M[0], n0, M[1], n1, M[2],
                         plan[2]);
      if (c1 <= kMaxSup) {
        const long long nc = (long long)nbt * c0 * n2;
        hipLaunchKernelGGL(axis_dft_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st,
                           box, vol, M[0], n0, n1, (long long)n2, M[1], nbt);
      } else {
        const long long nb1 = (n2 + kLines - 1) / kLines;
        hipLaunchKernelGGL(fft_strided_kernel, dim3((unsigned)(c0 * nb1), nbt), dim3(256),
                           lds_bytes(n1), st, box, vol, M[0], n0, (long long)n2, M[1], plan[1]);
      }
      const long long inner0 = (long long)n1 * n2;
      if (c0 <= kMaxSup) {
        const long long nc = (long long)nbt * inner0;
        hipLaunchKernelGGL(axis_dft_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st,
                           box, vol, -1, 1, n0, inner0, M[0], nbt);
      } else {
        hipLaunchKernelGGL(fft_strided_kernel,
                           dim3((unsigned)((inner0 + kLines - 1) / kLines), nbt), dim3(256),
                           lds_bytes(n0), st, box, vol, -1, 1, inner0, M[0], plan[0]);
      }
      if (psi_pts) {
        const long long nt = (long long)nbt * npts;
        hipLaunchKernelGGL(interp_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st,
                           box, vol, n0, n1, n2, d_base, d_w, d_ph, d_order, npts, nbt,
                           psi_pts + ((size_t)k * nb + b0) * npts);
      } else {
        const long long nt = (long long)nbt * vol;
        hipLaunchKernelGGL(grid_out_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st,
                           box, vol, n0, n1, n2, d_ph, iso, nbt,
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
