// Per-site dielectric solve in the radial x real-Y_lm basis (Sec. VI.E) and its adjoint.
//
// For a site with n_rad shells r_i (weights u_i) and n_ang directions (weights w_a):
//   X_{(L,i),(L',j)} = sum_{a,b} w_a Y_L(a) chi0(i a, j b) Y_L'(b) w_b
//   V_L(i,j) = 4 pi/(2l+1) min(r_i,r_j)^l / max(r_i,r_j)^(l+1)      (Coulomb, diagonal in L)
//   eps = I - V D X D,  W = eps^-1 V                                  (D = diag(u_i))
// solved per site by Gauss-Jordan elimination with partial pivoting on [eps | V] in FP64.
// Adjoint: dL/dX = D W^T Gbar W^T D,  dL/dchi0 = P^T (dL/dX) P.
// Induced density and potential of a spherical perturbation v1 (in the L = 00 channel):
//   y = (I - V D X D)^-1 v1 (the total potential),  rho = X D y,  v_ind = y - v1,
// which equal rho = (I - X D V D)^-1 X D v1 = chi D v1 and v_ind = V D rho (push-through);
// optionally with the 00;00 block alone (the l = 0 response).
// ALDA vertex (App. ALDA, Eqs. chi-alda and kxc_alda): with the contact kernel f_xc(n(r)),
// F_{(L,i),(L',i)} = sum_a w_a Y_L(a) f_xc(r_i a) Y_L'(a), the ALDA polarizability gives
//   W~ = V + V D X D Y,  Y = (I - V D X D - F X D)^-1 V.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "lrs_internal.h"

namespace lrs {
namespace {

// per-site metadata (device): offsets into the packed tables and buffers
struct SiteMeta {
  int nrad, nang, nL, n;        // n = nL * nrad
  int rad_off, yw_off;          // into radii/u and the Y*w table
  long long chi_off;            // site block offset in the site-block chi0 layout (npts^2)
  long long w_off;              // offset of the site's n x n matrices (W, X, T, ...)
  long long pt_off;             // first site point (for rho)
  long long h_off;              // offset of the site's length-n vectors
};

struct ScreenTabs {
  const SiteMeta* meta;
  const double* radii;
  const double* u;
  const double* yw;             // [sum nL * nang] : w_a Y_L(a), row L
};

__device__ inline double coulomb_l(int l, double ri, double rj) {
  double lo = fmin(ri, rj), hi = fmax(ri, rj);
  double v = 4.0 * 3.14159265358979323846 / (2 * l + 1) / hi;
  for (int k = 0; k < l; ++k) v *= lo / hi;
  return v;
}

__device__ inline int l_of(int L) { return L == 0 ? 0 : (L < 4 ? 1 : 2); }

// X block (i, j) of one site: one workgroup per (site, i, j)
__global__ void project_kernel(ScreenTabs T, const int4* blocks, const double* chi0,
                               double* X) {
  __shared__ double t1[9 * kMaxDirections];   // nL x nang
  const int4 bk = blocks[blockIdx.x];
  const SiteMeta m = T.meta[bk.x];
  const int i = bk.y, j = bk.z, A = m.nang, nL = m.nL;
  const int npts = m.nrad * A;
  const double* yw = T.yw + m.yw_off;
  const double* c = chi0 + m.chi_off + (long long)(i * A) * npts + j * A;
  for (int it = threadIdx.x; it < nL * A; it += blockDim.x) {
    const int L = it / A, b = it % A;
    double s = 0;
    for (int a = 0; a < A; ++a) s += yw[L * A + a] * c[(long long)a * npts + b];
    t1[L * A + b] = s;
  }
  __syncthreads();
  for (int it = threadIdx.x; it < nL * nL; it += blockDim.x) {
    const int L = it / nL, Lp = it % nL;
    double s = 0;
    for (int b = 0; b < A; ++b) s += t1[L * A + b] * yw[Lp * A + b];
    X[m.w_off + (long long)(L * m.nrad + i) * m.n + Lp * m.nrad + j] = s;
  }
}

// augmented [eps | V] rows: one workgroup per (site, row)
__global__ void eps_kernel(ScreenTabs T, const int2* rows, const double* X, double* M) {
  const int2 rw = rows[blockIdx.x];
  const SiteMeta m = T.meta[rw.x];
  const int row = rw.y, n = m.n, R = m.nrad;
  const int L = row / R, i = row % R, l = l_of(L);
  const double* r = T.radii + m.rad_off;
  const double* u = T.u + m.rad_off;
  const double* x = X + m.w_off;
  double* out = M + 2 * m.w_off + row;   // column-major: element (row, c) at c * n
  for (int c = threadIdx.x; c < 2 * n; c += blockDim.x) {
    if (c < n) {
      const int j = c % R;
      double s = 0;
      for (int q = 0; q < R; ++q) s += coulomb_l(l, r[i], r[q]) * u[q] * x[(long long)(L * R + q) * n + c];
      out[(long long)c * n] = (c == row ? 1.0 : 0.0) - s * u[j];
    } else {
      const int cc = c - n, Lp = cc / R, j = cc % R;
      out[(long long)c * n] = Lp == L ? coulomb_l(l, r[i], r[j]) : 0.0;
    }
  }
}

// Gauss-Jordan with partial pivoting on the augmented matrix of one site, stored column-major
// at M + 2 w_off (column c at c * n, n rows):
//   mode 0: [eps | V], 2n columns; the right block (W) goes to out + w_out_off[site], row-major
//   mode 1: [eps | v1], n + 1 columns; the last column (y) goes to out + h_off
//   mode 2: as 1 on the 00;00 block (n_rad rows)
// One workgroup of 1024 threads per site, blocked by panels of GJ_NB columns.  The panel is
// eliminated in LDS, wave w owning panel column w: at each step the owner of the step's column
// finds and swaps in the pivot, then every other wave swaps the same rows in its column (the
// multipliers of earlier steps included, so that they end up in the final row order) and the
// later columns are eliminated; the step's column keeps its multipliers.  Then every later column is read once, in the panel's
// final row order, takes the panel's nb elimination steps in registers and is written back
// (a wave updates four columns at a time, sharing the multipliers read from LDS).  The columns
// left of the panel are unit vectors by then and are not touched again.
// SLOTS 64-row slots of each column in registers: 5 (n <= 320) or 7 (n <= kMaxBasis; a few
// registers then spill, so sites that fit take the smaller form)
constexpr int GJ_NB = 16, GJ_COLS = 4;
static_assert(7 * 64 >= kMaxBasis, "the larger form holds every basis");
static_assert(64 % GJ_NB == 0, "a panel's rows must lie in one 64-row slot");
static_assert(1024 / 64 >= GJ_NB, "one wave per panel column");

__device__ __forceinline__ double gj_readlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The panel's nb elimination steps on GJ_COLS columns held in registers, row lane + 64 t in
// x[.][t].  Panels start at multiples of GJ_NB, so the panel's rows lie in one slot S of every
// column: the pivot-row value of step k is a read of lane (j0 + k) % 64 of x[.][S], and only
// slot S needs the pivot-row case.
template <int S, int SLOTS>
__device__ __forceinline__ void gj_panel_steps(double (&x)[GJ_COLS][SLOTS],
                                               const double (*pan)[SLOTS * 64], const double* inv_s,
                                               int j0, int nb, int n, int lane) {
  for (int k = 0; k < nb; ++k) {
    const int col = j0 + k, l = col & 63;
    const double inv = inv_s[k];
    double xp[GJ_COLS];
#pragma unroll
    for (int q = 0; q < GJ_COLS; ++q) xp[q] = gj_readlane(x[q][S], l) * inv;
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
      const int r = lane + 64 * t;
      const double f = r < n ? pan[k][r] : 0.0;
#pragma unroll
      for (int q = 0; q < GJ_COLS; ++q) {
        const double v = x[q][t] - f * xp[q];
        x[q][t] = (t == S && lane == l) ? xp[q] : v;
      }
    }
  }
}

template <int SLOTS>
__global__ void __launch_bounds__(1024) gauss_jordan_kernel(ScreenTabs T, double* M, int mode,
                                                            double* out,
                                                            const long long* w_out_off) {
  constexpr int GJ_MAXN = SLOTS * 64;
  __shared__ double pan[GJ_NB][GJ_MAXN];
  __shared__ int perm[GJ_MAXN];
  __shared__ double inv_s[GJ_NB];
  __shared__ int piv_s;
  const SiteMeta m = T.meta[blockIdx.x];
  const int n = mode == 2 ? m.nrad : m.n, n2 = n + (mode == 0 ? n : 1);
  double* A = M + 2 * m.w_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int j0 = 0; j0 < n; j0 += GJ_NB) {
    const int nb = min(GJ_NB, n - j0);
    for (int it = tid; it < nb * n; it += blockDim.x) {
      const int k = it / n, r = it - k * n;
      pan[k][r] = A[(long long)(j0 + k) * n + r];
    }
    for (int r = tid; r < n; r += blockDim.x) perm[r] = r;
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
      const int col = j0 + k;
      if (wave == k) {
        // pivot: the largest |pan[k][r]| for r >= col (lowest row on ties), swapped into place
        double best = -1.0;
        int bi = col;
        for (int r = col + lane; r < n; r += 64) {
          const double v = fabs(pan[k][r]);
          if (v > best) { best = v; bi = r; }
        }
        for (int o = 32; o > 0; o >>= 1) {
          const double ov = __shfl_xor(best, o);
          const int oi = __shfl_xor(bi, o);
          if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
        }
        if (lane == 0) {
          if (bi != col) {
            const double t = pan[k][col];
            pan[k][col] = pan[k][bi];
            pan[k][bi] = t;
            const int pt = perm[col];
            perm[col] = perm[bi];
            perm[bi] = pt;
          }
          piv_s = bi;
          inv_s[k] = 1.0 / pan[k][col];
        }
      }
      __syncthreads();
      // wave w owns panel column w: the same row swap (the multipliers of earlier steps
      // included), then for later columns the elimination of column col and the scaling of
      // the pivot-row entry.  Within a wave the LDS accesses keep program order.
      if (wave < nb && wave != k) {
        const int p = piv_s;
        if (p != col && lane == 0) {
          const double t = pan[wave][col];
          pan[wave][col] = pan[wave][p];
          pan[wave][p] = t;
        }
        if (wave > k) {
          const double piv = pan[wave][col] * inv_s[k];
          for (int r = lane; r < n; r += 64)
            if (r != col) pan[wave][r] -= pan[k][r] * piv;
          if (lane == 0) pan[wave][col] = piv;
        }
      }
      __syncthreads();
    }
    __syncthreads();
    // the later columns, GJ_COLS per wave at a time
    const int c0 = j0 + nb;
    for (int g = c0 + wave * GJ_COLS; g < n2; g += nw * GJ_COLS) {
      double x[GJ_COLS][SLOTS];
#pragma unroll
      for (int q = 0; q < GJ_COLS; ++q)
#pragma unroll
        for (int t = 0; t < SLOTS; ++t) {
          const int r = lane + 64 * t;
          x[q][t] = (g + q < n2 && r < n) ? A[(long long)(g + q) * n + perm[r]] : 0.0;
        }
      switch (j0 >> 6) {
        case 0: gj_panel_steps<0, SLOTS>(x, pan, inv_s, j0, nb, n, lane); break;
        case 1: gj_panel_steps<1, SLOTS>(x, pan, inv_s, j0, nb, n, lane); break;
        case 2: gj_panel_steps<2, SLOTS>(x, pan, inv_s, j0, nb, n, lane); break;
        case 3: gj_panel_steps<3, SLOTS>(x, pan, inv_s, j0, nb, n, lane); break;
        case 4: gj_panel_steps<4, SLOTS>(x, pan, inv_s, j0, nb, n, lane); break;
        case 5:
          if constexpr (SLOTS > 5) gj_panel_steps<5, SLOTS>(x, pan, inv_s, j0, nb, n, lane);
          break;
        default:
          if constexpr (SLOTS > 6) gj_panel_steps<6, SLOTS>(x, pan, inv_s, j0, nb, n, lane);
          break;
      }
#pragma unroll
      for (int q = 0; q < GJ_COLS; ++q)
#pragma unroll
        for (int t = 0; t < SLOTS; ++t) {
          const int r = lane + 64 * t;
          if (g + q < n2 && r < n) A[(long long)(g + q) * n + r] = x[q][t];
        }
    }
    __syncthreads();
  }
  if (mode == 0) {
    double* W = out + w_out_off[blockIdx.x];
    for (int it = tid; it < n * n; it += blockDim.x) {
      const int c = it / n, r = it - c * n;
      W[(long long)r * n + c] = A[(long long)(n + c) * n + r];
    }
  } else {
    for (int r = tid; r < n; r += blockDim.x) out[m.h_off + r] = A[(long long)n * n + r];
  }
}

// augmented [eps | v1] rows of the induced-potential solve: one workgroup per (site, row);
// l0: the 00;00 block only (rows and columns L = 00).  v1 [sum n_rad]: the radial values.
__global__ void induced_rows_kernel(ScreenTabs T, const int2* rows, const double* X,
                                    const double* v1, int l0, double* M) {
  const int2 rw = rows[blockIdx.x];
  const SiteMeta m = T.meta[rw.x];
  const int row = rw.y, R = m.nrad, n = m.n;
  const int sz = l0 ? R : n;
  if (row >= sz) return;
  const int L = row / R, i = row % R, l = l_of(L);
  const double* r = T.radii + m.rad_off;
  const double* u = T.u + m.rad_off;
  const double* x = X + m.w_off;
  double* out = M + 2 * m.w_off + row;   // column-major: element (row, c) at c * sz
  for (int c = threadIdx.x; c <= sz; c += blockDim.x) {
    if (c < sz) {
      const int j = c % R;
      double acc = 0;
      for (int q = 0; q < R; ++q) acc += coulomb_l(l, r[i], r[q]) * u[q] * x[(long long)(L * R + q) * n + c];
      out[(long long)c * sz] = (c == row ? 1.0 : 0.0) - acc * u[j];
    } else {
      // the Y_00 coefficient of the spherical v1
      out[(long long)c * sz] = L == 0 ? 2.0 * sqrt(3.14159265358979323846) * v1[m.rad_off + i] : 0.0;
    }
  }
}

// rho = X D y and v_ind = y - v1 for one site (one workgroup per site)
__global__ void induced_out_kernel(ScreenTabs T, const double* X, const double* y,
                                   const double* v1, int l0, double* rho, double* vind) {
  const SiteMeta m = T.meta[blockIdx.x];
  const int R = m.nrad, n = m.n, sz = l0 ? R : n;
  const double* x = X + m.w_off;
  const double* u = T.u + m.rad_off;
  const double* yy = y + m.h_off;
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    double rr = 0.0, vv = 0.0;
    if (r < sz) {
      for (int c = 0; c < sz; ++c) rr += x[(long long)r * n + c] * u[c % R] * yy[c];
      const double v1r = r < R ? 2.0 * sqrt(3.14159265358979323846) * v1[m.rad_off + r] : 0.0;
      vv = yy[r] - v1r;
    }
    rho[m.h_off + r] = rr;
    vind[m.h_off + r] = vv;
  }
}

// ---- valence W(x, x') inside r_m (Sec. V.A, Eq. rpa-val): every site is a grid point x with the
// induced potential v_ind of a uniformly charged sphere of radius R_x (unit charge) on its shells.
struct ValenceArgs {
  const double* vind;    // [sum n] induced potential, (L, i) L-major per site (at h_off)
  const double* centre;  // [nsites][3]
  double cell[9], inv[9];   // lattice vectors (rows) and the inverse transpose; has_cell = 0: none
  int has_cell, nsites, nL;
  double R_x, r_shell, eps_inf, r_m;
  double* W;             // [nsites][nsites]
};

__device__ inline void real_ylm_dev(double x, double y, double z, double* Y) {
  const double pi = 3.14159265358979323846;
  const double c1 = sqrt(3.0 / (4.0 * pi)), c2 = sqrt(15.0 / (4.0 * pi));
  const double c20 = sqrt(5.0 / (16.0 * pi));
  Y[0] = 0.5 / sqrt(pi);
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  Y[4] = c2 * x * y;
  Y[5] = c2 * y * z;
  Y[6] = c20 * (3.0 * z * z - 1.0);
  Y[7] = c2 * x * z;
  Y[8] = 0.5 * c2 * (x * x - y * y);
}

// cubic Lagrange interpolation of f (stride `stride`, nr samples at radii r) at x: the four
// shells nearest to x, clamped at the ends of the grid
__device__ inline double lagrange4_dev(const double* r, const double* f, int nr, double x) {
  int i = 0;
  while (i < nr && r[i] < x) ++i;
  i = min(max(i - 2, 0), nr - 4);
  double out = 0.0;
  for (int a = 0; a < 4; ++a) {
    double w = 1.0;
    for (int b = 0; b < 4; ++b)
      if (b != a) w *= (x - r[i + b]) / (r[i + a] - r[i + b]);
    out += w * f[i + a];
  }
  return out;
}

__device__ inline double sphere_pot(double r, double R) {
  return r < R ? (3.0 - r * r / (R * R)) / (2.0 * R) : 1.0 / r;
}

// W^[a](centre_a + d)
__device__ double valence_one_way(const ScreenTabs& T, const ValenceArgs& A, int a, double dx,
                                  double dy, double dz) {
  const SiteMeta m = T.meta[a];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  double Y[9];
  real_ylm_dev(dx / r, dy / r, dz / r, Y);
  const double* rad = T.radii + m.rad_off;
  double v = sphere_pot(r, A.R_x);
  for (int L = 0; L < A.nL; ++L)
    v += Y[L] * lagrange4_dev(rad, A.vind + m.h_off + (long long)L * m.nrad, m.nrad, r);
  const double v2 = r < A.r_shell ? 1.0 / A.r_shell : 1.0 / r;
  return v - (1.0 - 1.0 / A.eps_inf) * v2;
}

// one thread per (a, b): W[a][b] = (W^[a](x_b) + W^[b](x_a)) / 2 within r_m (the same two terms
// in both orders, so W is exactly symmetric), the discretisation-sphere average on the
// diagonal, zero beyond r_m
__global__ void valence_pairs_kernel(ScreenTabs T, ValenceArgs A) {
  const int a = blockIdx.y * blockDim.y + threadIdx.y;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A.nsites || b >= A.nsites) return;
  double* out = A.W + (long long)a * A.nsites + b;
  if (a == b) {
    // (3 / R^3) int_0^R W_00(r) r^2 dr: the bare sphere 6 / (5 R), the shell's v2 (constant
    // inside R_S > R), the induced l = 0 part by 8-point Gauss-Legendre on [0, R]
    const double gx[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                          -0.1834346424956498, 0.1834346424956498, 0.5255324099163290,
                          0.7966664774136267, 0.9602898564975363};
    const double gw[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                          0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                          0.2223810344533745, 0.1012285362903763};
    const SiteMeta m = T.meta[a];
    const double* rad = T.radii + m.rad_off;
    const double R = A.R_x;
    double s = 0.0;
    for (int q = 0; q < 8; ++q) {
      const double r = 0.5 * R * (gx[q] + 1.0);
      s += 0.5 * R * gw[q] * r * r * lagrange4_dev(rad, A.vind + m.h_off, m.nrad, r);
    }
    const double y00 = 0.5 / sqrt(3.14159265358979323846);
    *out = 6.0 / (5.0 * R) + 3.0 / (R * R * R) * y00 * s - (1.0 - 1.0 / A.eps_inf) / A.r_shell;
    return;
  }
  double d[3];
  for (int c = 0; c < 3; ++c) d[c] = A.centre[3 * b + c] - A.centre[3 * a + c];
  if (A.has_cell) {
    // nearest periodic image: subtract the rounded fractional coordinates
    double f[3];
    for (int c = 0; c < 3; ++c) f[c] = rint(A.inv[3 * c] * d[0] + A.inv[3 * c + 1] * d[1] + A.inv[3 * c + 2] * d[2]);
    for (int c = 0; c < 3; ++c) d[c] -= f[0] * A.cell[c] + f[1] * A.cell[3 + c] + f[2] * A.cell[6 + c];
  }
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (r > A.r_m) {
    *out = 0.0;
    return;
  }
  *out = 0.5 * (valence_one_way(T, A, a, d[0], d[1], d[2]) +
                valence_one_way(T, A, b, -d[0], -d[1], -d[2]));
}

// ---- ALDA: the LDA exchange-correlation energy per volume, e(n) = n (eps_x + eps_c), with
// Slater exchange eps_x = -(3/4) (3n/pi)^(1/3) and the Vosko-Wilk-Nusair (1980) paramagnetic
// correlation (fit to Ceperley-Alder; Hartree units), x = sqrt(r_s), X(x) = x^2 + b x + c
__device__ double lda_energy(double n) {
  const double pi = 3.14159265358979323846;
  const double A = 0.0310907, x0 = -0.10498, b = 3.72744, c = 12.9352;
  const double ex = -0.75 * cbrt(3.0 * n / pi);
  const double rs = cbrt(3.0 / (4.0 * pi * n));
  const double x = sqrt(rs);
  const double Q = sqrt(4.0 * c - b * b);
  const double X = x * x + b * x + c, X0 = x0 * x0 + b * x0 + c;
  const double at = atan(Q / (2.0 * x + b));
  const double ec = A * (log(x * x / X) + 2.0 * b / Q * at -
                         b * x0 / X0 * (log((x - x0) * (x - x0) / X) + 2.0 * (b + 2.0 * x0) / Q * at));
  return n * (ex + ec);
}

// f_xc = d^2 e / dn^2 at every site point: 5-point central difference with density steps of
// 0.01, shrunk to n/4 where n < 0.04 so that every stencil density stays positive; 0 for n <= 0
__global__ void fxc_kernel(const double* dens, long long npts, double* f) {
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts;
       p += (long long)gridDim.x * blockDim.x) {
    const double n = dens[p];
    double v = 0.0;
    if (n > 0.0) {
      const double h = fmin(0.01, 0.25 * n);
      v = (-lda_energy(n + 2 * h) + 16.0 * lda_energy(n + h) - 30.0 * lda_energy(n) +
           16.0 * lda_energy(n - h) - lda_energy(n - 2 * h)) / (12.0 * h * h);
    }
    f[p] = v;
  }
}

// contact matrix F[(i, L, L')] = sum_a w_a Y_L(a) f(r_i a) Y_L'(a) of one (site, shell); the
// unweighted Y_L'(a) is yw[L'][a] / w_a with w_a = 2 sqrt(pi) yw[0][a]
__global__ void contact_kernel(ScreenTabs T, const double* f, double* F) {
  const SiteMeta m = T.meta[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= m.nrad) return;
  const int nL = m.nL, A = m.nang;
  const double* yw = T.yw + m.yw_off;
  const double* fi = f + m.pt_off + (long long)i * A;
  double* out = F + (long long)m.h_off * nL + (long long)i * nL * nL;
  for (int it = threadIdx.x; it < nL * nL; it += blockDim.x) {
    const int L = it / nL, Lp = it % nL;
    double acc = 0;
    for (int a = 0; a < A; ++a)
      acc += yw[L * A + a] * yw[Lp * A + a] * fi[a] / (2.0 * sqrt(3.14159265358979323846) * yw[a]);
    out[it] = acc;
  }
}

// augmented [I - V D X D - F X D | V] rows: one workgroup per (site, row)
__global__ void alda_rows_kernel(ScreenTabs T, const int2* rows, const double* X,
                                 const double* F, double* M) {
  const int2 rw = rows[blockIdx.x];
  const SiteMeta m = T.meta[rw.x];
  const int row = rw.y, n = m.n, R = m.nrad, nL = m.nL;
  const int L = row / R, i = row % R, l = l_of(L);
  const double* r = T.radii + m.rad_off;
  const double* u = T.u + m.rad_off;
  const double* x = X + m.w_off;
  const double* fi = F + (long long)m.h_off * nL + (long long)i * nL * nL + L * nL;
  double* out = M + 2 * m.w_off + row;   // column-major: element (row, c) at c * n
  for (int c = threadIdx.x; c < 2 * n; c += blockDim.x) {
    if (c < n) {
      const int j = c % R;
      double acc = 0;
      for (int q = 0; q < R; ++q) acc += coulomb_l(l, r[i], r[q]) * u[q] * x[(long long)(L * R + q) * n + c];
      for (int Lp = 0; Lp < nL; ++Lp) acc += fi[Lp] * x[(long long)(Lp * R + i) * n + c];
      out[(long long)c * n] = (c == row ? 1.0 : 0.0) - acc * u[j];
    } else {
      const int cc = c - n, Lp = cc / R, j = cc % R;
      out[(long long)c * n] = Lp == L ? coulomb_l(l, r[i], r[j]) : 0.0;
    }
  }
}

// T = X D Y (pass 1) and W~ = V + V D T (pass 2); grid (row, site), threads over columns
__global__ void alda_pass1(ScreenTabs T, const double* X, const double* Y, double* Tm) {
  const SiteMeta m = T.meta[blockIdx.y];
  const int n = m.n, R = m.nrad, rr = blockIdx.x;
  if (rr >= n) return;
  const double* x = X + m.w_off + (long long)rr * n;
  const double* y = Y + m.w_off;
  const double* u = T.u + m.rad_off;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double acc = 0;
    for (int k = 0; k < n; ++k) acc += x[k] * u[k % R] * y[(long long)k * n + c];
    Tm[m.w_off + (long long)rr * n + c] = acc;
  }
}

__global__ void alda_pass2(ScreenTabs T, const double* Tm, double* W_out,
                           const long long* w_out_off) {
  const SiteMeta m = T.meta[blockIdx.y];
  const int n = m.n, R = m.nrad, rr = blockIdx.x;
  if (rr >= n) return;
  const int L = rr / R, i = rr % R, l = l_of(L);
  const double* r = T.radii + m.rad_off;
  const double* u = T.u + m.rad_off;
  const double* t = Tm + m.w_off;
  double* W = W_out + w_out_off[blockIdx.y] + (long long)rr * n;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int Lp = c / R, j = c % R;
    double acc = Lp == L ? coulomb_l(l, r[i], r[j]) : 0.0;
    for (int q = 0; q < R; ++q) acc += coulomb_l(l, r[i], r[q]) * u[q] * t[(long long)(L * R + q) * n + c];
    W[c] = acc;
  }
}

// rho_L = P rho and h = D rho_L for one site; optional loss h^T W h
__global__ void charge_kernel(ScreenTabs T, const double* rho, const double* W,
                              const long long* w_out_off, double* h_out, double* loss) {
  __shared__ double h[kMaxBasis + 32];
  __shared__ double part[1024 / 64];
  const SiteMeta m = T.meta[blockIdx.x];
  const int R = m.nrad, A = m.nang, n = m.n;
  const double* yw = T.yw + m.yw_off;
  const double* u = T.u + m.rad_off;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const int L = q / R, i = q % R;
    double s = 0;
    for (int a = 0; a < A; ++a) s += yw[L * A + a] * rho[m.pt_off + (long long)i * A + a];
    h[q] = s * u[i];
    h_out[m.h_off + q] = s * u[i];
  }
  __syncthreads();
  if (!loss) return;
  const double* w = W + w_out_off[blockIdx.x];
  double acc = 0;
  for (long long it = threadIdx.x; it < (long long)n * n; it += blockDim.x) {
    const int r = (int)(it / n), c = (int)(it % n);
    acc += h[r] * w[it] * h[c];
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) s += part[w2];
    loss[blockIdx.x] = s;
  }
}

// dX = D (W^T G W^T) D for one site; G = dL/dW, or h h^T when dLdW is NULL.
// Two passes through small tiles: T1 = W^T G, then dX = T1 W^T.
__global__ void wtgw_pass1(ScreenTabs T, const double* W, const long long* w_out_off,
                           const double* G, const double* h, double* T1, int rank_one) {
  // grid: (site, row tile) ; each thread a column
  const int site = blockIdx.y;
  const SiteMeta m = T.meta[site];
  const int n = m.n;
  const int r = blockIdx.x;
  if (r >= n) return;
  const double* w = W + w_out_off[site];
  const double* g = G ? G + w_out_off[site] : nullptr;
  const double* hv = h + m.h_off;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double s = 0;
    if (rank_one) {
      // (W^T h h^T)[r][c] = (sum_q W[q][r] h[q]) h[c]
      for (int q = 0; q < n; ++q) s += w[(long long)q * n + r] * hv[q];
      s *= hv[c];
    } else {
      for (int q = 0; q < n; ++q) s += w[(long long)q * n + r] * g[(long long)q * n + c];
    }
    T1[m.w_off + (long long)r * n + c] = s;
  }
}

__global__ void wtgw_pass2(ScreenTabs T, const double* W, const long long* w_out_off,
                           const double* T1, double* dX) {
  const int site = blockIdx.y;
  const SiteMeta m = T.meta[site];
  const int n = m.n, R = m.nrad;
  const int r = blockIdx.x;
  if (r >= n) return;
  const double* w = W + w_out_off[site];
  const double* u = T.u + m.rad_off;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double s = 0;
    for (int q = 0; q < n; ++q) s += T1[m.w_off + (long long)r * n + q] * w[(long long)c * n + q];
    dX[m.w_off + (long long)r * n + c] = s * u[r % R] * u[c % R];
  }
}

// dL/dchi0 block (i, j) = sum_{L,L'} yw[L][a] dX[(L,i),(L',j)] yw[L'][b]
__global__ void lambda_kernel(ScreenTabs T, const int4* blocks, const double* dX, double* out) {
  __shared__ double u1[9 * kMaxDirections];
  __shared__ double dxb[81];
  const int4 bk = blocks[blockIdx.x];
  const SiteMeta m = T.meta[bk.x];
  const int i = bk.y, j = bk.z, A = m.nang, nL = m.nL, R = m.nrad, n = m.n;
  const int npts = R * A;
  const double* yw = T.yw + m.yw_off;
  for (int it = threadIdx.x; it < nL * nL; it += blockDim.x) {
    const int L = it / nL, Lp = it % nL;
    dxb[it] = dX[m.w_off + (long long)(L * R + i) * n + Lp * R + j];
  }
  __syncthreads();
  for (int it = threadIdx.x; it < nL * A; it += blockDim.x) {
    const int L = it / A, b = it % A;
    double s = 0;
    for (int Lp = 0; Lp < nL; ++Lp) s += dxb[L * nL + Lp] * yw[Lp * A + b];
    u1[L * A + b] = s;
  }
  __syncthreads();
  double* o = out + m.chi_off + (long long)(i * A) * npts + j * A;
  for (int it = threadIdx.x; it < A * A; it += blockDim.x) {
    const int a = it / A, b = it % A;
    double s = 0;
    for (int L = 0; L < nL; ++L) s += yw[L * A + a] * u1[L * A + b];
    o[(long long)a * npts + b] = s;
  }
}

// real spherical harmonics, l <= 2, order L = l*l + l + m
void real_ylm(double x, double y, double z, double* Y) {
  const double pi = 3.14159265358979323846;
  const double c0 = 0.5 / std::sqrt(pi);
  const double c1 = std::sqrt(3.0 / (4.0 * pi));
  const double c2 = std::sqrt(15.0 / (4.0 * pi));
  const double c20 = std::sqrt(5.0 / (16.0 * pi));
  Y[0] = c0;
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  Y[4] = c2 * x * y;
  Y[5] = c2 * y * z;
  Y[6] = c20 * (3.0 * z * z - 1.0);
  Y[7] = c2 * x * z;
  Y[8] = 0.5 * c2 * (x * x - y * y);
}

struct HostTabs {
  std::vector<SiteMeta> meta;
  std::vector<double> radii, u, yw;
  std::vector<int4> blocks;
  std::vector<int2> rows;
  std::vector<long long> w_out_off;
  long long w_total = 0;   // sum n^2
  long long n_total = 0;   // sum n
  int max_n = 0;
};

void build_tabs(const lrs_ctx* ctx, HostTabs& H) {
  const int nL = (ctx->lmax + 1) * (ctx->lmax + 1);
  long long chi = 0, w = 0, ywo = 0;
  for (int s = 0; s < ctx->nsites; ++s) {
    SiteMeta m;
    m.nrad = ctx->nrad[s];
    m.nang = ctx->nang[s];
    m.nL = nL;
    m.n = nL * m.nrad;
    m.rad_off = ctx->rad_off[s];
    m.yw_off = (int)ywo;
    m.chi_off = chi;
    m.w_off = w;
    m.pt_off = ctx->site_off[s];
    m.h_off = H.n_total;
    H.meta.push_back(m);
    H.w_out_off.push_back(w);
    for (int L = 0; L < nL; ++L)
      for (int a = 0; a < m.nang; ++a) {
        const double* p = &ctx->ang_xyz[3 * (size_t)(ctx->ang_off[s] + a)];
        double Y[9];
        real_ylm(p[0], p[1], p[2], Y);
        H.yw.push_back(Y[L] * ctx->ang_w[ctx->ang_off[s] + a]);
      }
    ywo += (long long)nL * m.nang;
    for (int i = 0; i < m.nrad; ++i)
      for (int j = 0; j < m.nrad; ++j) H.blocks.push_back(make_int4(s, i, j, 0));
    for (int r = 0; r < m.n; ++r) H.rows.push_back(make_int2(s, r));
    chi += (long long)m.nrad * m.nang * m.nrad * m.nang;
    w += (long long)m.n * m.n;
    H.n_total += m.n;
    H.max_n = std::max(H.max_n, m.n);
  }
  H.w_total = w;
  H.radii = ctx->radii;
  H.u = ctx->rad_w;
}

// device layout of screen_tab: meta | radii | u | yw | blocks | rows | w_out_off
struct DevTabs {
  ScreenTabs t;
  const int4* blocks;
  const int2* rows;
  const long long* w_out_off;
  int nblocks, nrows;
};

hipError_t upload_tabs(lrs_ctx* ctx, const HostTabs& H, DevTabs& D) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  size_t o_meta = take(H.meta.size() * sizeof(SiteMeta));
  size_t o_rad = take(H.radii.size() * 8), o_u = take(H.u.size() * 8), o_yw = take(H.yw.size() * 8);
  size_t o_blk = take(H.blocks.size() * sizeof(int4)), o_rows = take(H.rows.size() * sizeof(int2));
  size_t o_wo = take(H.w_out_off.size() * 8);
  if (ctx->screen_tab.bytes < off) {
    if (ctx->screen_tab.p) {
      (void)hipFree(ctx->screen_tab.p);
      ctx->bytes_in_use -= ctx->screen_tab.bytes;
      ctx->screen_tab.p = nullptr;
      ctx->screen_tab.bytes = 0;
    }
    hipError_t e = hipMalloc(&ctx->screen_tab.p, off);
    if (e != hipSuccess) return e;
    ctx->screen_tab.bytes = off;
    ctx->bytes_in_use += off;
  }
  char* b = (char*)ctx->screen_tab.p;
  hipStream_t s = ctx->stream;
  hipError_t e = hipSuccess;
  auto put = [&](size_t o, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(b + o, src, bytes, hipMemcpyHostToDevice, s);
  };
  put(o_meta, H.meta.data(), H.meta.size() * sizeof(SiteMeta));
  put(o_rad, H.radii.data(), H.radii.size() * 8);
  put(o_u, H.u.data(), H.u.size() * 8);
  put(o_yw, H.yw.data(), H.yw.size() * 8);
  put(o_blk, H.blocks.data(), H.blocks.size() * sizeof(int4));
  put(o_rows, H.rows.data(), H.rows.size() * sizeof(int2));
  put(o_wo, H.w_out_off.data(), H.w_out_off.size() * 8);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // host tables are freed on return
  D.t.meta = (const SiteMeta*)(b + o_meta);
  D.t.radii = (const double*)(b + o_rad);
  D.t.u = (const double*)(b + o_u);
  D.t.yw = (const double*)(b + o_yw);
  D.blocks = (const int4*)(b + o_blk);
  D.rows = (const int2*)(b + o_rows);
  D.w_out_off = (const long long*)(b + o_wo);
  D.nblocks = (int)H.blocks.size();
  D.nrows = (int)H.rows.size();
  return e;
}

hipError_t ensure_dev(lrs_ctx* ctx, DevBuf& b, size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  if (b.p && b.bytes >= bytes) return hipSuccess;
  if (b.p) {
    (void)hipFree(b.p);
    ctx->bytes_in_use -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  if (ctx->max_bytes && ctx->bytes_in_use + bytes > ctx->max_bytes) return hipErrorOutOfMemory;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    return hipErrorOutOfMemory;
  }
  b.bytes = bytes;
  ctx->bytes_in_use += bytes;
  return hipSuccess;
}

}  // namespace

// work layout: X [w_total] | M [2 w_total] | h [n_total]; W_last [w_total]; rho_last [nrows]
hipError_t launch_screen_forward(lrs_ctx* ctx, const double* chi0_ss, double* W_out,
                                 const double* rho, double* loss_out) {
  HostTabs H;
  build_tabs(ctx, H);
  if (H.max_n > kMaxBasis) return hipErrorInvalidValue;
  for (const auto& m : H.meta)
    if (m.nang > kMaxDirections) return hipErrorInvalidValue;
  DevTabs D;
  hipError_t e = upload_tabs(ctx, H, D);
  if (e != hipSuccess) return e;
  e = ensure_dev(ctx, ctx->work, (size_t)(3 * H.w_total + H.n_total) * 8);
  if (e == hipSuccess) e = ensure_dev(ctx, ctx->W_last, (size_t)H.w_total * 8);
  if (e == hipSuccess && rho) e = ensure_dev(ctx, ctx->rho_last, (size_t)ctx->nrows * 8);
  if (e != hipSuccess) return e;
  double* X = (double*)ctx->work.p;
  double* M = X + H.w_total;
  double* h = M + 2 * H.w_total;
  hipLaunchKernelGGL(project_kernel, dim3(D.nblocks), dim3(256), 0, ctx->stream, D.t, D.blocks,
                     chi0_ss, X);
  hipLaunchKernelGGL(eps_kernel, dim3(D.nrows), dim3(256), 0, ctx->stream, D.t, D.rows, X, M);
  hipLaunchKernelGGL(H.max_n <= 320 ? gauss_jordan_kernel<5> : gauss_jordan_kernel<7>,
                     dim3(ctx->nsites), dim3(1024), 0, ctx->stream, D.t, M,
                     0, W_out, D.w_out_off);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(ctx->W_last.p, W_out, (size_t)H.w_total * 8, hipMemcpyDeviceToDevice,
                     ctx->stream);
  if (e != hipSuccess) return e;
  ctx->have_rho = false;
  if (rho) {
    e = hipMemcpyAsync(ctx->rho_last.p, rho, (size_t)ctx->nrows * 8, hipMemcpyDeviceToDevice,
                       ctx->stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(charge_kernel, dim3(ctx->nsites), dim3(256), 0, ctx->stream, D.t, rho,
                       W_out, D.w_out_off, h, loss_out);
    ctx->have_rho = true;
  }
  ctx->have_W = true;
  return hipGetLastError();
}

hipError_t launch_screen_backward(lrs_ctx* ctx, const double* dL_dW, double* dL_dchi0) {
  HostTabs H;
  build_tabs(ctx, H);
  DevTabs D;
  hipError_t e = upload_tabs(ctx, H, D);
  if (e != hipSuccess) return e;
  double* X = (double*)ctx->work.p;     // reused as T1 and dX
  double* M = X + H.w_total;
  double* h = M + 2 * H.w_total;
  double* T1 = X;
  double* dX = M;
  const double* W = (const double*)ctx->W_last.p;
  if (!dL_dW) {
    hipLaunchKernelGGL(charge_kernel, dim3(ctx->nsites), dim3(256), 0, ctx->stream, D.t,
                       (const double*)ctx->rho_last.p, W, D.w_out_off, h, (double*)nullptr);
  }
  dim3 grid(H.max_n, ctx->nsites);
  hipLaunchKernelGGL(wtgw_pass1, grid, dim3(256), 0, ctx->stream, D.t, W, D.w_out_off, dL_dW, h,
                     T1, dL_dW ? 0 : 1);
  hipLaunchKernelGGL(wtgw_pass2, grid, dim3(256), 0, ctx->stream, D.t, W, D.w_out_off, T1, dX);
  hipLaunchKernelGGL(lambda_kernel, dim3(D.nblocks), dim3(256), 0, ctx->stream, D.t, D.blocks, dX,
                     dL_dchi0);
  return hipGetLastError();
}

// work layout: X [w_total] | M [2 w_total] | y [n_total] | v1 [sum n_rad]
static hipError_t launch_induced(lrs_ctx* ctx, const double* chi0_ss, const double* v1_host, int l0,
                          double* rho_out, double* v_out) {
  HostTabs H;
  build_tabs(ctx, H);
  if (H.max_n > kMaxBasis) return hipErrorInvalidValue;
  for (const auto& m : H.meta)
    if (m.nang > kMaxDirections) return hipErrorInvalidValue;
  DevTabs D;
  hipError_t e = upload_tabs(ctx, H, D);
  if (e != hipSuccess) return e;
  const size_t nrad_total = H.radii.size();
  e = ensure_dev(ctx, ctx->work, (size_t)(3 * H.w_total + H.n_total + nrad_total) * 8);
  if (e != hipSuccess) return e;
  double* X = (double*)ctx->work.p;
  double* M = X + H.w_total;
  double* y = M + 2 * H.w_total;
  double* v1 = y + H.n_total;
  e = hipMemcpyAsync(v1, v1_host, nrad_total * 8, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);   // v1_host may be a temporary
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(project_kernel, dim3(D.nblocks), dim3(256), 0, ctx->stream, D.t, D.blocks,
                     chi0_ss, X);
  hipLaunchKernelGGL(induced_rows_kernel, dim3(D.nrows), dim3(256), 0, ctx->stream, D.t, D.rows,
                     X, v1, l0, M);
  hipLaunchKernelGGL(H.max_n <= 320 ? gauss_jordan_kernel<5> : gauss_jordan_kernel<7>,
                     dim3(ctx->nsites), dim3(1024), 0, ctx->stream, D.t, M,
                     l0 ? 2 : 1, y, D.w_out_off);
  hipLaunchKernelGGL(induced_out_kernel, dim3(ctx->nsites), dim3(256), 0, ctx->stream, D.t, X, y,
                     v1, l0, rho_out, v_out);
  return hipGetLastError();
}

// work layout: X [w_total] | M [2 w_total] | Y [w_total] | T [w_total] | F [n_total nL] |
// f [nrows]
static hipError_t launch_alda(lrs_ctx* ctx, const double* chi0_ss, const double* dens,
                              double* W_out) {
  HostTabs H;
  build_tabs(ctx, H);
  if (H.max_n > kMaxBasis) return hipErrorInvalidValue;
  for (const auto& m : H.meta)
    if (m.nang > kMaxDirections) return hipErrorInvalidValue;
  DevTabs D;
  hipError_t e = upload_tabs(ctx, H, D);
  if (e != hipSuccess) return e;
  const int nL = (ctx->lmax + 1) * (ctx->lmax + 1);
  e = ensure_dev(ctx, ctx->work,
                 (size_t)(5 * H.w_total + H.n_total * nL + (long long)ctx->nrows) * 8);
  if (e != hipSuccess) return e;
  double* X = (double*)ctx->work.p;
  double* M = X + H.w_total;
  double* Y = M + 2 * H.w_total;
  double* Tm = Y + H.w_total;
  double* F = Tm + H.w_total;
  double* f = F + H.n_total * nL;
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(fxc_kernel, dim3(256), dim3(256), 0, st, dens, (long long)ctx->nrows, f);
  hipLaunchKernelGGL(contact_kernel, dim3(H.max_n / nL, ctx->nsites), dim3(64), 0, st, D.t, f, F);
  hipLaunchKernelGGL(project_kernel, dim3(D.nblocks), dim3(256), 0, st, D.t, D.blocks, chi0_ss, X);
  hipLaunchKernelGGL(alda_rows_kernel, dim3(D.nrows), dim3(256), 0, st, D.t, D.rows, X, F, M);
  hipLaunchKernelGGL(H.max_n <= 320 ? gauss_jordan_kernel<5> : gauss_jordan_kernel<7>,
                     dim3(ctx->nsites), dim3(1024), 0, st, D.t, M, 0, Y,
                     D.w_out_off);
  dim3 grid(H.max_n, ctx->nsites);
  hipLaunchKernelGGL(alda_pass1, grid, dim3(256), 0, st, D.t, X, Y, Tm);
  hipLaunchKernelGGL(alda_pass2, grid, dim3(256), 0, st, D.t, Tm, W_out, D.w_out_off);
  return hipGetLastError();
}

// Valence W of the sites as grid points: the induced potential of the sphere's v1 at every site
// (the induced-potential solve, full response), then the pair kernel.
// val_work layout: rho [n_total] | v_ind [n_total] | centres [3 nsites]
static hipError_t launch_valence(lrs_ctx* ctx, const double* chi0_ss, const double* centres,
                                 const double* cell, double vx, double r_shell, double eps_inf,
                                 double r_m, double* W_out) {
  const double pi = 3.14159265358979323846;
  const double R_x = std::cbrt(3.0 * vx / (4.0 * pi));
  std::vector<double> v1(ctx->radii.size());
  for (size_t i = 0; i < v1.size(); ++i) {
    const double r = ctx->radii[i];
    const double ve = r < R_x ? (3.0 - r * r / (R_x * R_x)) / (2.0 * R_x) : 1.0 / r;
    v1[i] = r < r_shell ? ve - 1.0 / r_shell : 0.0;     // v_ext - v2 (zero beyond the shell)
  }
  HostTabs H;
  build_tabs(ctx, H);
  hipError_t e = ensure_dev(ctx, ctx->val_work, (size_t)(2 * H.n_total + 3 * ctx->nsites) * 8);
  if (e != hipSuccess) return e;
  double* rho = (double*)ctx->val_work.p;
  double* vind = rho + H.n_total;
  double* cen = vind + H.n_total;
  e = hipMemcpyAsync(cen, centres, (size_t)3 * ctx->nsites * 8, hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) return e;
  e = launch_induced(ctx, chi0_ss, v1.data(), 0, rho, vind);   // synchronises (host tables)
  if (e != hipSuccess) return e;
  DevTabs D;
  e = upload_tabs(ctx, H, D);
  if (e != hipSuccess) return e;
  ValenceArgs A;
  A.vind = vind;
  A.centre = cen;
  A.has_cell = cell != nullptr;
  for (int i = 0; i < 9; ++i) A.cell[i] = cell ? cell[i] : 0.0;
  if (cell) {
    // inverse of the transpose: fractional coordinates f = A^-T d, row c of `inv` gives f_c
    const double* a = cell;
    const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                       a[2] * (a[3] * a[7] - a[4] * a[6]);
    // adjugate of A (rows a1, a2, a3): (A^-1)_{ij}; f_c = sum_j (A^-T)_{cj} d_j = sum_j (A^-1)_{jc} d_j
    double ai[9];
    ai[0] = (a[4] * a[8] - a[5] * a[7]) / det;
    ai[1] = (a[2] * a[7] - a[1] * a[8]) / det;
    ai[2] = (a[1] * a[5] - a[2] * a[4]) / det;
    ai[3] = (a[5] * a[6] - a[3] * a[8]) / det;
    ai[4] = (a[0] * a[8] - a[2] * a[6]) / det;
    ai[5] = (a[2] * a[3] - a[0] * a[5]) / det;
    ai[6] = (a[3] * a[7] - a[4] * a[6]) / det;
    ai[7] = (a[1] * a[6] - a[0] * a[7]) / det;
    ai[8] = (a[0] * a[4] - a[1] * a[3]) / det;
    for (int c = 0; c < 3; ++c)
      for (int j = 0; j < 3; ++j) A.inv[3 * c + j] = ai[3 * j + c];
  }
  A.nsites = ctx->nsites;
  A.nL = (ctx->lmax + 1) * (ctx->lmax + 1);
  A.R_x = R_x;
  A.r_shell = r_shell;
  A.eps_inf = eps_inf;
  A.r_m = r_m;
  A.W = W_out;
  const dim3 blk(16, 16), grd((ctx->nsites + 15) / 16, (ctx->nsites + 15) / 16);
  hipLaunchKernelGGL(valence_pairs_kernel, grd, blk, 0, ctx->stream, D.t, A);
  return hipGetLastError();
}

// Host-side check of the solve kernels' limits: n = (lmax+1)^2 n_rad <= kMaxBasis basis
// functions (the Gauss-Jordan kernel's register slots) and at most kMaxDirections directions
// per site (the projection's LDS table).
bool screen_sizes_ok(const lrs_ctx* ctx) {
  const int nL = (ctx->lmax + 1) * (ctx->lmax + 1);
  for (int s = 0; s < ctx->nsites; ++s)
    if (nL * ctx->nrad[s] > kMaxBasis || ctx->nang[s] > kMaxDirections) return false;
  return true;
}

}  // namespace lrs

using namespace lrs;

extern "C" lrs_status lrs_screen_W_alda(lrs_ctx* ctx, const double* chi0_sitesite,
                                        const double* density, double* W_out) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (!ctx->have_sites) {
    ctx->err = "sites must be set first";
    return LRS_ESTATE;
  }
  if (!chi0_sitesite || !density || !W_out) {
    ctx->err = "missing argument";
    return LRS_EINVAL;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipSetDevice(ctx->device) != hipSuccess ||
      hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess) {
    ctx->err = "device";
    return LRS_EDEVICE;
  }
  if (cs != hipStreamCaptureStatusNone) {
    ctx->err = "the ALDA solve copies host tables; it cannot be captured";
    return LRS_ESTATE;
  }
  if (!screen_sizes_ok(ctx)) {
    ctx->err = "a site basis exceeds 448 functions or 256 directions";
    return LRS_EUNSUPPORTED;
  }
  const hipError_t e = launch_alda(ctx, chi0_sitesite, density, W_out);
  if (e == hipErrorOutOfMemory) {
    ctx->err = "ALDA workspace";
    return LRS_ENOMEM;
  }
  if (e != hipSuccess) {
    ctx->err = std::string("ALDA W: ") + hipGetErrorString(e);
    return LRS_EDEVICE;
  }
  return LRS_OK;
}

extern "C" lrs_status lrs_induced_potential(lrs_ctx* ctx, const double* chi0_sitesite,
                                            const double* v1_host, double q, double r_shell,
                                            int l0_only, double* rho_out, double* v_out) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (!ctx->have_sites) {
    ctx->err = "sites must be set first";
    return LRS_ESTATE;
  }
  if (!chi0_sitesite || !rho_out || !v_out) {
    ctx->err = "missing argument";
    return LRS_EINVAL;
  }
  std::vector<double> v1(ctx->radii.size());
  if (v1_host) {
    for (size_t i = 0; i < v1.size(); ++i) {
      if (!std::isfinite(v1_host[i])) {
        ctx->err = "v1 must be finite";
        return LRS_ENONFINITE;
      }
      v1[i] = v1_host[i];
    }
  } else {
    if (!std::isfinite(q) || !(r_shell > 0) || !std::isfinite(r_shell)) {
      ctx->err = "q must be finite and r_shell positive";
      return LRS_EINVAL;
    }
    // short-range part of q / r after the shell partition: q (1/r - 1/R_S) inside the shell
    for (size_t i = 0; i < v1.size(); ++i) {
      const double r = ctx->radii[i];
      v1[i] = r < r_shell ? q * (1.0 / r - 1.0 / r_shell) : 0.0;
    }
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipSetDevice(ctx->device) != hipSuccess ||
      hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess) {
    ctx->err = "device";
    return LRS_EDEVICE;
  }
  if (cs != hipStreamCaptureStatusNone) {
    ctx->err = "the induced-potential solve copies host tables; it cannot be captured";
    return LRS_ESTATE;
  }
  if (!screen_sizes_ok(ctx)) {
    ctx->err = "a site basis exceeds 448 functions or 256 directions";
    return LRS_EUNSUPPORTED;
  }
  const hipError_t e = launch_induced(ctx, chi0_sitesite, v1.data(), l0_only != 0, rho_out, v_out);
  if (e == hipErrorOutOfMemory) {
    ctx->err = "induced-potential workspace";
    return LRS_ENOMEM;
  }
  if (e != hipSuccess) {
    ctx->err = std::string("induced potential: ") + hipGetErrorString(e);
    return LRS_EDEVICE;
  }
  return LRS_OK;
}

extern "C" lrs_status lrs_valence_W(lrs_ctx* ctx, const double* chi0_sitesite,
                                    const double* centres_host, const double* cell_host, double vx,
                                    double r_shell, double eps_inf, double r_m, double* W_out) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (!ctx->have_sites) {
    ctx->err = "sites must be set first";
    return LRS_ESTATE;
  }
  if (!chi0_sitesite || !centres_host || !W_out) {
    ctx->err = "missing argument";
    return LRS_EINVAL;
  }
  for (int i = 0; i < 3 * ctx->nsites; ++i)
    if (!std::isfinite(centres_host[i])) {
      ctx->err = "non-finite site centre";
      return LRS_ENONFINITE;
    }
  if (cell_host)
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(cell_host[i])) {
        ctx->err = "non-finite lattice vector";
        return LRS_ENONFINITE;
      }
  const double R_x = std::cbrt(3.0 * vx / (4.0 * 3.14159265358979323846));
  if (!(vx > 0) || !std::isfinite(vx) || !(r_shell > R_x) || !std::isfinite(r_shell) ||
      !(eps_inf >= 1.0) || !std::isfinite(eps_inf) || !(r_m > 0) || !std::isfinite(r_m)) {
    ctx->err = "need vx > 0, r_shell > R_x = (3 vx / 4 pi)^(1/3), eps_inf >= 1 and r_m > 0";
    return LRS_EINVAL;
  }
  if (cell_host) {
    const double* a = cell_host;
    const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                       a[2] * (a[3] * a[7] - a[4] * a[6]);
    if (!(std::fabs(det) > 0)) {
      ctx->err = "singular lattice";
      return LRS_EINVAL;
    }
  }
  for (int s = 0; s < ctx->nsites; ++s) {
    const int nr = ctx->nrad[s];
    if (nr < 4) {
      ctx->err = "every site needs at least 4 shells (cubic radial interpolation)";
      return LRS_EUNSUPPORTED;
    }
    if (ctx->radii[ctx->rad_off[s] + nr - 1] < r_m) {
      ctx->err = "r_m exceeds a site's largest shell radius";
      return LRS_EINVAL;
    }
  }
  if (!screen_sizes_ok(ctx)) {
    ctx->err = "a site basis exceeds 448 functions or 256 directions";
    return LRS_EUNSUPPORTED;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipSetDevice(ctx->device) != hipSuccess ||
      hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess) {
    ctx->err = "device";
    return LRS_EDEVICE;
  }
  if (cs != hipStreamCaptureStatusNone) {
    ctx->err = "the valence assembly copies host tables; it cannot be captured";
    return LRS_ESTATE;
  }
  const hipError_t e = launch_valence(ctx, chi0_sitesite, centres_host, cell_host, vx, r_shell,
                                      eps_inf, r_m, W_out);
  if (e == hipErrorOutOfMemory) {
    ctx->err = "valence workspace";
    return LRS_ENOMEM;
  }
  if (e != hipSuccess) {
    ctx->err = std::string("valence W: ") + hipGetErrorString(e);
    return LRS_EDEVICE;
  }
  return LRS_OK;
}

// ------------------------------------------------------------------ allocation-free W solve
// lrs_screen_W_noalloc runs the kernels of lrs_screen_W with its tables and workspace in this
// fixed device array instead of context buffers.  Every GPU the library runs on holds its own
// copy until the process ends.  Host code must never pass the array's name to a kernel or a
// copy (in host code it is a stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returned for the current device, kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[lrs::kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

namespace lrs {

// Looks up the scratch array's address on `device` (which must be current); once per device.
hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

namespace {

// Scratch layout of one call: meta | radii | u | yw | blocks | rows | w_out_off, then
// X [w_total] | M [2 w_total] | h [n_total] (the workspace of lrs_screen_W).  Returns the bytes
// needed; with base != null also fills D and the workspace pointers.
size_t noalloc_layout(const HostTabs& H, unsigned char* base, DevTabs* D, double** X,
                      double** M, double** h, size_t* offs) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  offs[0] = take(H.meta.size() * sizeof(SiteMeta));
  offs[1] = take(H.radii.size() * 8);
  offs[2] = take(H.u.size() * 8);
  offs[3] = take(H.yw.size() * 8);
  offs[4] = take(H.blocks.size() * sizeof(int4));
  offs[5] = take(H.rows.size() * sizeof(int2));
  offs[6] = take(H.w_out_off.size() * 8);
  const size_t o_x = take((size_t)H.w_total * 8);
  const size_t o_m = take((size_t)2 * H.w_total * 8);
  const size_t o_h = take((size_t)H.n_total * 8);
  if (base) {
    D->t.meta = (const SiteMeta*)(base + offs[0]);
    D->t.radii = (const double*)(base + offs[1]);
    D->t.u = (const double*)(base + offs[2]);
    D->t.yw = (const double*)(base + offs[3]);
    D->blocks = (const int4*)(base + offs[4]);
    D->rows = (const int2*)(base + offs[5]);
    D->w_out_off = (const long long*)(base + offs[6]);
    D->nblocks = (int)H.blocks.size();
    D->nrows = (int)H.rows.size();
    *X = (double*)(base + o_x);
    *M = (double*)(base + o_m);
    *h = (double*)(base + o_h);
  }
  return off;
}

}  // namespace
}  // namespace lrs

extern "C" lrs_status lrs_screen_W_noalloc(lrs_ctx* ctx, const double* chi0_sitesite,
                                           double* W_out, const double* rho_test,
                                           double* loss_out) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (!ctx->have_sites) {
    ctx->err = "sites must be set first";
    return LRS_ESTATE;
  }
  if (!chi0_sitesite || !W_out) {
    ctx->err = "chi0 and W_out are required";
    return LRS_EINVAL;
  }
  if (loss_out && !rho_test) {
    ctx->err = "loss_out needs rho_test";
    return LRS_EINVAL;
  }
  if (!screen_sizes_ok(ctx)) {
    ctx->err = "a site basis exceeds 448 functions or 256 directions";
    return LRS_EUNSUPPORTED;
  }
  HostTabs H;
  build_tabs(ctx, H);
  size_t offs[7];
  const size_t need = noalloc_layout(H, nullptr, nullptr, nullptr, nullptr, nullptr, offs);
  if (need > kScratchBytes) {
    char buf[160];
    snprintf(buf, sizeof(buf), "the solve needs %zu bytes of scratch; the fixed array holds %zu",
             need, kScratchBytes);
    ctx->err = buf;
    return LRS_ENOMEM;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipSetDevice(ctx->device) != hipSuccess ||
      hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess) {
    ctx->err = "device";
    return LRS_EDEVICE;
  }
  if (cs != hipStreamCaptureStatusNone) {
    ctx->err = "the solve copies host tables into its scratch; it cannot be captured";
    return LRS_ESTATE;
  }
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices)
      base = (unsigned char*)g_scratch_ptr[ctx->device];
  }
  if (!base) {
    ctx->err = "the scratch array's address on this device was not set up";
    return LRS_EDEVICE;
  }
  DevTabs D;
  double *X = nullptr, *M = nullptr, *h = nullptr;
  noalloc_layout(H, base, &D, &X, &M, &h, offs);
  hipStream_t st = ctx->stream;
  hipError_t e = hipSuccess;
  auto put = [&](size_t o, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(base + o, src, bytes, hipMemcpyHostToDevice, st);
  };
  put(offs[0], H.meta.data(), H.meta.size() * sizeof(SiteMeta));
  put(offs[1], H.radii.data(), H.radii.size() * 8);
  put(offs[2], H.u.data(), H.u.size() * 8);
  put(offs[3], H.yw.data(), H.yw.size() * 8);
  put(offs[4], H.blocks.data(), H.blocks.size() * sizeof(int4));
  put(offs[5], H.rows.data(), H.rows.size() * sizeof(int2));
  put(offs[6], H.w_out_off.data(), H.w_out_off.size() * 8);
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host tables die on return
  if (e == hipSuccess) {
    // X, M and h are written in full by the kernels before they are read: nothing to clear
    hipLaunchKernelGGL(project_kernel, dim3(D.nblocks), dim3(256), 0, st, D.t, D.blocks,
                       chi0_sitesite, X);
    hipLaunchKernelGGL(eps_kernel, dim3(D.nrows), dim3(256), 0, st, D.t, D.rows, X, M);
    hipLaunchKernelGGL(H.max_n <= 320 ? gauss_jordan_kernel<5> : gauss_jordan_kernel<7>,
                     dim3(ctx->nsites), dim3(1024), 0, st, D.t, M, 0,
                       W_out, D.w_out_off);
    if (rho_test)
      hipLaunchKernelGGL(charge_kernel, dim3(ctx->nsites), dim3(256), 0, st, D.t, rho_test,
                         W_out, D.w_out_off, h, loss_out);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    ctx->err = std::string("screen_W_noalloc: ") + hipGetErrorString(e);
    return LRS_EDEVICE;
  }
  return LRS_OK;
}
