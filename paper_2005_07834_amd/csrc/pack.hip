// Operand packing: complex128 orbitals -> the matrix-core fragment layouts used by the chi0
// kernels, plus small helpers (max |x|, zero fill).
//
// The contraction index K runs over (k-point, band) pairs: occupied pairs first
// ([0, Ko), k-major), zeros up to Ko_pad, then unoccupied pairs ([Ko_pad, Ko_pad + Ku)),
// zeros up to K_pad.  Padding is zero so that padded products vanish.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include "lrs_internal.h"

namespace lrs {
namespace {

struct SrcPsi {           // complex128 [nk][nb][ld] orbitals on a point set
  const double* psi;
  int nb, nocc, nu, ncols, ld, Ko, Ko_pad, Ku;
  // real orbitals: slot k of a 16-slot chunk c holds orbital K = 32 c + k%16 as its re value
  // and K + 16 as its im value, each orbital's real part (Ko_pad then counts orbitals, twice
  // the slots)
  int real;
  __device__ const double* at(int c, int k) const {   // orbital k's value at c, or null
    int kp, band;
    if (k < Ko) {
      kp = k / nocc;
      band = k - kp * nocc;
    } else if (k >= Ko_pad && k < Ko_pad + Ku) {
      int j = k - Ko_pad;
      kp = j / nu;
      band = nocc + (j - kp * nu);
    } else {
      return nullptr;
    }
    return psi + 2 * ((size_t)(kp * nb + band) * ld + c);
  }
  __device__ void get(int c, int k, double& re, double& im) const {
    re = 0.0;
    im = 0.0;
    if (c >= ncols) return;
    if (real) {
      const int K = 32 * (k >> 4) + (k & 15);
      const double* a = at(c, K);
      const double* b = at(c, K + 16);
      re = a ? a[0] : 0.0;
      im = b ? b[0] : 0.0;
      return;
    }
    const double* p = at(c, k);
    if (!p) return;
    re = p[0];
    im = p[1];
  }
};

struct SrcTiles64 {       // FP64 fragment tiles as a source (for lazy reduced-precision copies)
  const double* t;
  int ncb;                // column blocks
  __device__ void get(int c, int k, double& re, double& im) const {
    int cb = c >> 4, ch = k >> 4, kl = k & 15;
    int lane = ((kl & 3) << 4) | (c & 15);
    int s = kl >> 2;
    const double* tile = t + ((size_t)ch * ncb + cb) * (kTileBytes / 8);
    re = tile[lane * 4 + s];
    im = tile[256 + lane * 4 + s];
  }
};

__device__ inline void split_bf16(float x, __hip_bfloat16& hi, __hip_bfloat16& lo) {
  hi = __float2bfloat16(x);
  lo = __float2bfloat16(x - __bfloat162float(hi));
}
__device__ inline void split_f16(float x, __half& hi, __half& lo) {
  hi = __float2half(x);
  lo = __float2half(x - __half2float(hi));
}

// One thread per (tile, lane slot): writes that slot of every plane of the tile.  Tiles are
// stored chunk-major: tile (column block cb, chunk ch) at index ch * ncb + cb, so that the
// blocks one workgroup needs for one chunk are contiguous.
//   FP64  (4 KiB, 64 slots):  slot l holds column l%16, k = 16 ch + 4 s + l/16, s = 0..3
//   FP32  (4 KiB, 64 slots):  slot l holds column l%16, k = 32 ch + 4 s + l/16, s = 0..7
//   split (2 KiB, 32 slots):  slot l holds column l%16, k = 16 ch + 8 (l/16) + e, e = 0..7,
//                             planes re hi, re lo, im hi, im lo
//   F16F8 (2 KiB, 32 slots): slot l holds column l%16, k = 16 ch + 8 (l/16) + e, e = 0..7:
//                             the fp16 hi slot of planes re and im and 8 bytes of each fp8
//                             plane (layout note in lrs_internal.h)
// F16F8 column operand: the 8 K values k0 .. k0 + 7 of column c (K half h of the chunk) go to
// fp16 hi slot 16 h + c of the re and im planes and to bytes 8 h .. 8 h + 7 of row c of the
// fp8 planes, part 0 = lo * 2^18 and part 1 = hi * 2^7 (the column side's order).
template <class Src>
__device__ void pack_f16f8_column(const Src& src, int c, int k0, float prescale,
                                  unsigned char* tile, int h) {
  _Float16 hr[8], hi_[8];
  unsigned int f8[4][2] = {};     // [re p0, re p1, im p0, im p1][dword]
  for (int j = 0; j < 8; ++j) {
    double re, im;
    src.get(c, k0 + j, re, im);
    const float xr = (float)(re * prescale), xi = (float)(im * prescale);
    const _Float16 a = (_Float16)xr, b = (_Float16)xi;
    hr[j] = a;
    hi_[j] = b;
    const float lr = xr - (float)a, li = xi - (float)b;
    const int sh = 8 * (j & 3), dw = j >> 2;
    f8[0][dw] |= e4m3_rn(ldexpf(lr, kF8LoShift)) << sh;
    f8[1][dw] |= e4m3_rn(ldexpf((float)a, kF8HiShift)) << sh;
    f8[2][dw] |= e4m3_rn(ldexpf(li, kF8LoShift)) << sh;
    f8[3][dw] |= e4m3_rn(ldexpf((float)b, kF8HiShift)) << sh;
  }
  _Float16* dr = reinterpret_cast<_Float16*>(tile + (16 * h + c % 16) * 16);
  _Float16* di = reinterpret_cast<_Float16*>(tile + 512 + (16 * h + c % 16) * 16);
  for (int e = 0; e < 8; ++e) {
    dr[e] = hr[e];
    di[e] = hi_[e];
  }
  for (int part = 0; part < 4; ++part) {
    uint2* d = reinterpret_cast<uint2*>(tile + 1024 + part * 256 + (c % 16) * 16 + 8 * h);
    *d = make_uint2(f8[part][0], f8[part][1]);
  }
}

template <class Src>
__global__ void pack_tiles_kernel(Src src, long long ntiles, int ncb, int prec,
                                  float prescale, unsigned char* out) {
  const bool split = prec == LRS_BF16X2 || prec == LRS_FP16X2 || prec == LRS_F16F8;
  const int slots = split ? 32 : 64;
  long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= ntiles * slots) return;
  int lane = (int)(gid % slots);
  long long tile = gid / slots;
  int ch = (int)(tile / ncb);
  int cb = (int)(tile - (long long)ch * ncb);
  int c = cb * 16 + (lane & 15);
  unsigned char* base = out + tile * (long long)tile_bytes(prec);
  if (prec == LRS_F16F8) {
    pack_f16f8_column(src, c, ch * 16 + 8 * (lane >> 4), prescale, base, lane >> 4);
  } else if (prec == LRS_FP64 || prec == LRS_FP64_3M) {
    // (3M: a third plane b_r + b_i, the column side's factor of the third product)
    double* t = reinterpret_cast<double*>(base);
    for (int s = 0; s < 4; ++s) {
      double re, im;
      src.get(c, ch * 16 + 4 * s + (lane >> 4), re, im);
      t[lane * 4 + s] = re;
      t[256 + lane * 4 + s] = im;
      if (prec == LRS_FP64_3M) t[512 + lane * 4 + s] = re + im;
    }
  } else if (prec == LRS_FP32) {
    float* t = reinterpret_cast<float*>(base);
    for (int s = 0; s < 8; ++s) {
      double re, im;
      src.get(c, ch * 32 + 4 * s + (lane >> 4), re, im);
      t[lane * 8 + s] = (float)re;
      t[512 + lane * 8 + s] = (float)im;
    }
  } else if (prec == LRS_BF16X2) {
    __hip_bfloat16* t = reinterpret_cast<__hip_bfloat16*>(base);
    for (int e = 0; e < 8; ++e) {
      double re, im;
      src.get(c, ch * 16 + 8 * (lane >> 4) + e, re, im);
      split_bf16((float)re, t[lane * 8 + e], t[256 + lane * 8 + e]);
      split_bf16((float)im, t[512 + lane * 8 + e], t[768 + lane * 8 + e]);
    }
  } else {
    __half* t = reinterpret_cast<__half*>(base);
    for (int e = 0; e < 8; ++e) {
      double re, im;
      src.get(c, ch * 16 + 8 * (lane >> 4) + e, re, im);
      split_f16((float)(re * prescale), t[lane * 8 + e], t[256 + lane * 8 + e]);
      split_f16((float)(im * prescale), t[512 + lane * 8 + e], t[768 + lane * 8 + e]);
    }
  }
}

// Site rows: planar [2][rows_pad][K_pad] FP64.  Within each 16-chunk of K the order is
// permuted (stored g*4 + j <-> k = 4 j + g) so that a lane's four FP64 matrix-core operands
// are contiguous.
__device__ inline size_t pos_f64(int r, int k, int K_pad) {
  int ch = k >> 4, kl = k & 15;
  return (size_t)r * K_pad + ch * 16 + (kl & 3) * 4 + (kl >> 2);
}

struct SrcSite64 {        // the FP64 row operand as a source (optionally through a column map)
  const double* a;
  int rows_pad, K_pad;
  const int* colmap;      // nullptr: identity
  __device__ void get(int r, int k, double& re, double& im) const {
    if (colmap) {
      r = colmap[r];
      if (r < 0) {
        re = 0.0;
        im = 0.0;
        return;
      }
    }
    size_t p = pos_f64(r, k, K_pad);
    re = a[p];
    im = a[(size_t)rows_pad * K_pad + p];
  }
};

__global__ void pack_site_rows_kernel(SrcPsi src, int rows_pad, int K_pad, double* o64) {
  long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long n = (long long)rows_pad * K_pad;
  if (gid >= n) return;
  int r = (int)(gid / K_pad);
  int k = (int)(gid - (long long)r * K_pad);
  double re, im;
  src.get(r, k, re, im);
  size_t p = pos_f64(r, k, K_pad);
  o64[p] = re;
  o64[(size_t)n + p] = im;
}

// Site orbitals k-major for the adjoint: planar [2][K_pad][rows_pad], natural K order.
__global__ void derive_site_kmajor_kernel(SrcSite64 src, double* out) {
  long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long n = (long long)src.rows_pad * src.K_pad;
  if (gid >= n) return;
  int k = (int)(gid / src.rows_pad);
  int r = (int)(gid - (long long)k * src.rows_pad);
  double re, im;
  src.get(r, k, re, im);
  out[gid] = re;
  out[n + gid] = im;
}

// real orbitals: orbital K (of 2 K_pad) is component (K / 16) % 2 of slot 16 (K / 32) + K % 16
__global__ void derive_site_kmajor_real_kernel(SrcSite64 src, double* out) {
  long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long n = 2LL * src.rows_pad * src.K_pad;
  if (gid >= n) return;
  int K = (int)(gid / src.rows_pad);
  int r = (int)(gid - (long long)K * src.rows_pad);
  double re, im;
  src.get(r, 16 * (K >> 5) + (K & 15), re, im);
  out[gid] = (K >> 4) & 1 ? im : re;
  out[n + gid] = 0.0;
}

// largest |Im| of n complex values (the odd doubles)
__global__ void max_abs_im_kernel(const double* x, long long n, unsigned int* out_bits) {
  float m = 0.f;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    m = fmaxf(m, (float)fabs(x[2 * i + 1]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out_bits, __float_as_uint(m));
}

__global__ void max_abs_kernel(const double* x, long long n, unsigned int* out_bits) {
  float m = 0.f;
  bool bad = false;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double v = x[i];
    if (!isfinite(v)) bad = true;
    m = fmaxf(m, (float)fabs(v));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  unsigned int any = __any(bad) ? 1u : 0u;
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out_bits, __float_as_uint(m));   // non-negative floats order like their bits
    if (any) atomicOr(out_bits + 1, 1u);
  }
}

__global__ void fill_zero_kernel(uint4* p, size_t n16) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0, 0, 0, 0);
}

inline int blocks_for(long long n, int tpb) { return (int)((n + tpb - 1) / tpb); }

}  // namespace

hipError_t launch_pack_tiles(const double* psi, int nk, int nb, int nocc, int ncols, int ld_src,
                             int ncols_pad, int Ko_pad, int K_pad, int prec, float prescale,
                             int real, void* out, hipStream_t s) {
  int nu = nb - nocc;
  SrcPsi src{psi, nb, nocc, nu, ncols, ld_src, nk * nocc, real ? 2 * Ko_pad : Ko_pad, nk * nu,
             real};
  int nchunks = K_pad / chunk_of(prec);
  long long ntiles = (long long)(ncols_pad / 16) * nchunks;
  hipLaunchKernelGGL(pack_tiles_kernel<SrcPsi>, dim3(blocks_for(ntiles * 64, 256)), dim3(256), 0,
                     s, src, ntiles, ncols_pad / 16, prec, prescale, (unsigned char*)out);
  return hipGetLastError();
}

hipError_t launch_repack_from_f64(const void* tiles64, int ncols_pad, int K_pad, int prec,
                                  float prescale, void* dst, hipStream_t s) {
  SrcTiles64 src{(const double*)tiles64, ncols_pad / 16};
  int nchunks = K_pad / chunk_of(prec);
  long long ntiles = (long long)(ncols_pad / 16) * nchunks;
  hipLaunchKernelGGL(pack_tiles_kernel<SrcTiles64>, dim3(blocks_for(ntiles * 64, 256)), dim3(256),
                     0, s, src, ntiles, ncols_pad / 16, prec, prescale, (unsigned char*)dst);
  return hipGetLastError();
}

hipError_t launch_pack_site_rows(const double* psi, int nk, int nb, int nocc, int nrows,
                                 int rows_pad, int Ko_pad, int K_pad, int real, double* out_f64,
                                 hipStream_t s) {
  int nu = nb - nocc;
  SrcPsi src{psi, nb, nocc, nu, nrows, nrows, nk * nocc, real ? 2 * Ko_pad : Ko_pad, nk * nu,
             real};
  long long n = (long long)rows_pad * K_pad;
  hipLaunchKernelGGL(pack_site_rows_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src,
                     rows_pad, K_pad, out_f64);
  return hipGetLastError();
}

hipError_t launch_derive_site_kmajor(const double* site_f64, int rows_pad, int K_pad, int real,
                                     double* out, hipStream_t s) {
  SrcSite64 src{site_f64, rows_pad, K_pad, nullptr};
  long long n = (long long)rows_pad * K_pad * (real ? 2 : 1);
  if (real)
    hipLaunchKernelGGL(derive_site_kmajor_real_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       src, out);
  else
    hipLaunchKernelGGL(derive_site_kmajor_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src,
                       out);
  return hipGetLastError();
}

hipError_t launch_site_col_tiles(const double* site_f64, int rows_pad, int K_pad, int ncols_pad,
                                 const int* colmap, int prec, float prescale, void* dst,
                                 hipStream_t s) {
  SrcSite64 src{site_f64, rows_pad, K_pad, colmap};
  int nchunks = K_pad / chunk_of(prec);
  long long ntiles = (long long)(ncols_pad / 16) * nchunks;
  hipLaunchKernelGGL(pack_tiles_kernel<SrcSite64>, dim3(blocks_for(ntiles * 64, 256)), dim3(256),
                     0, s, src, ntiles, ncols_pad / 16, prec, prescale, (unsigned char*)dst);
  return hipGetLastError();
}

hipError_t launch_max_abs(const double* x, long long n, unsigned int* out_bits, hipStream_t s) {
  int blocks = (int)std::min<long long>(4096, std::max<long long>(1, (n + 255) / 256));
  hipLaunchKernelGGL(max_abs_kernel, dim3(blocks), dim3(256), 0, s, x, n, out_bits);
  return hipGetLastError();
}

hipError_t launch_max_abs_im(const double* psi, long long n, unsigned int* out_bits,
                             hipStream_t s) {
  int blocks = (int)std::min<long long>(4096, std::max<long long>(1, (n + 255) / 256));
  hipLaunchKernelGGL(max_abs_im_kernel, dim3(blocks), dim3(256), 0, s, psi, n, out_bits);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  int blocks = (int)std::min<size_t>(8192, (n16 + 255) / 256);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, (uint4*)p, n16);
  return hipGetLastError();
}

}  // namespace lrs
