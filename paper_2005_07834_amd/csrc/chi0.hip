// chi0 on the matrix cores (Sec. VI.D with the energy quadrature of Appendix D.1.b).
//
// For one output tile (rows r of the site operand x columns r' of the column operand) and
// each quadrature term l, a workgroup forms the two weighted Green's function tiles
//     G_o^l(r,r') = sum_{K occ}   conj(psi_K(r)) alpha_l(K) psi_K(r')
//     G_u^l(r,r') = sum_{K unocc} conj(psi_K(r)) beta_l(K)  psi_K(r')
// as complex GEMMs in the real 4M form (G_r = p b_r + q b_i, G_i = p b_i - q b_r with
// p + i q = weight * psi(r)) on MFMA, then accumulates
//     chi(r,r') += c_l (Re G_o Re G_u + Im G_o Im G_u)
// in FP64 registers.  After the last term the tile is scaled by -2 s / N_k^2 and stored.
//
// The per-term weight is applied to the small site operand while it is staged into LDS, so
// the large column operand is identical for every term.  BF16X2 / FP16X2 split the weighted
// site value into hi + lo halves on the fly; the column operand is pre-split.  Each real
// product takes hi*hi + hi*lo + lo*hi (lo*lo dropped) with FP32 accumulation.
//
// Persistent launch: gridDim.x workgroups walk a host-built tile list; workgroup b handles
// tiles b' + i * gridDim.x with b' = (b % 8) * (gridDim.x / 8) + b / 8, so that the
// workgroups resident on one XCD (dispatch is round-robin over the 8 XCDs) take a contiguous
// run of the list, which the host orders in 8 x 8 groups of (row tile, column tile): the
// concurrently running workgroups of an XCD share operand tiles in that XCD's L2.
#include <hip/hip_runtime.h>

#include "lrs_internal.h"

namespace lrs {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned int)))) unsigned int u32x4;

struct Chi0Params {
  const void* a_re;
  const void* a_im;
  int lda;                      // = K_pad (row stride of the site operand and of the weights)
  const unsigned char* b;       // column operand fragment tiles [colblock][chunk][4 KiB]
  int b_nchunks;
  const void* w;                // weights [T][K_pad]
  const double* c;              // [T]
  int T, nch_o, nch_u;
  const TileDesc* tiles;
  int ntiles;
  double* out;
  double pref;
  float a_scale;                // power-of-two prescale of the site operand (FP16X2)
  // adjoint mode (FP64 only): with T = 1, write lam * conj(G_u) and lam * conj(G_o)
  const double* lam;
  double* hu_re;
  double* hu_im;
  double* ho_re;
  double* ho_im;
};

template <int PREC>
struct Prec;
template <>
struct Prec<LRS_FP64> {
  using acc_t = f64x4;
  using site_t = double;
  static constexpr int KC = 16;
};
template <>
struct Prec<LRS_FP32> {
  using acc_t = f32x4;
  using site_t = float;
  static constexpr int KC = 32;
};
template <>
struct Prec<LRS_BF16X2> {
  using acc_t = f32x4;
  using site_t = float;
  static constexpr int KC = 32;
};
template <>
struct Prec<LRS_FP16X2> {
  using acc_t = f32x4;
  using site_t = float;
  static constexpr int KC = 32;
};

// ----------------------------------------------------------------------------- staging
// Site operand: item (row r, lane group g) covers the K values one lane of the 16-row block
// holds; the row operand's chunk-local order makes them contiguous (see pack.hip).
template <int PREC>
__device__ __forceinline__ void stage_a_item(const Chi0Params& P, unsigned char* lds_a, int r,
                                             int g, int a_row, int t, int kbase) {
  const int blk = r >> 4;
  const int slot = g * 16 + (r & 15);
  unsigned char* base = lds_a + blk * kTileBytes;
  if constexpr (PREC == LRS_FP64) {
    const double* are = (const double*)P.a_re + (size_t)a_row * P.lda + kbase + g * 4;
    const double* aim = (const double*)P.a_im + (size_t)a_row * P.lda + kbase + g * 4;
    const double* wt = (const double*)P.w + (size_t)t * P.lda + kbase + g * 4;
    f64x4 re = *(const f64x4*)are, im = *(const f64x4*)aim, w = *(const f64x4*)wt;
    *(f64x4*)(base + slot * 32) = re * w;
    *(f64x4*)(base + 2048 + slot * 32) = im * w;
  } else if constexpr (PREC == LRS_FP32) {
    const float* are = (const float*)P.a_re + (size_t)a_row * P.lda + kbase + g * 8;
    const float* aim = (const float*)P.a_im + (size_t)a_row * P.lda + kbase + g * 8;
    const float* wt = (const float*)P.w + (size_t)t * P.lda + kbase + g * 8;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f32x4 re = *(const f32x4*)(are + 4 * h), im = *(const f32x4*)(aim + 4 * h),
            w = *(const f32x4*)(wt + 4 * h);
      *(f32x4*)(base + slot * 32 + 16 * h) = re * w;
      *(f32x4*)(base + 2048 + slot * 32 + 16 * h) = im * w;
    }
  } else {
    const float* are = (const float*)P.a_re + (size_t)a_row * P.lda + kbase + g * 8;
    const float* aim = (const float*)P.a_im + (size_t)a_row * P.lda + kbase + g * 8;
    const float* wt = (const float*)P.w + (size_t)t * P.lda + kbase + g * 8;
    using half_t = typename std::conditional<PREC == LRS_BF16X2, bf16x8, f16x8>::type;
    using elem_t = typename std::conditional<PREC == LRS_BF16X2, __bf16, _Float16>::type;
    half_t ph, pl, qh, ql;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f32x4 re = *(const f32x4*)(are + 4 * h), im = *(const f32x4*)(aim + 4 * h),
            w = *(const f32x4*)(wt + 4 * h);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float p = re[e] * w[e] * P.a_scale;
        float q = im[e] * w[e] * P.a_scale;
        elem_t phe = (elem_t)p, qhe = (elem_t)q;
        ph[4 * h + e] = phe;
        qh[4 * h + e] = qhe;
        pl[4 * h + e] = (elem_t)(p - (float)phe);
        ql[4 * h + e] = (elem_t)(q - (float)qhe);
      }
    }
    *(half_t*)(base + slot * 16) = ph;
    *(half_t*)(base + 1024 + slot * 16) = pl;
    *(half_t*)(base + 2048 + slot * 16) = qh;
    *(half_t*)(base + 3072 + slot * 16) = ql;
  }
}

// ----------------------------------------------------------------------------- MFMA step
template <int PREC, int MB, int NB>
__device__ __forceinline__ void mma_chunk(const unsigned char* lds_a, const unsigned char* lds_b,
                                          int lane,
                                          typename Prec<PREC>::acc_t (&gr)[MB][NB],
                                          typename Prec<PREC>::acc_t (&gi)[MB][NB]) {
  if constexpr (PREC == LRS_FP64) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double p[MB], q[MB];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        p[i] = ((const double*)(lds_a + i * kTileBytes))[lane * 4 + s];
        q[i] = ((const double*)(lds_a + i * kTileBytes + 2048))[lane * 4 + s];
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        double br = ((const double*)(lds_b + j * kTileBytes))[lane * 4 + s];
        double bi = ((const double*)(lds_b + j * kTileBytes + 2048))[lane * 4 + s];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
          gr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(p[i], br, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(q[i], bi, gr[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(p[i], bi, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-q[i], br, gi[i][j], 0, 0, 0);
        }
      }
    }
  } else if constexpr (PREC == LRS_FP32) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f32x4 p[MB], q[MB];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        p[i] = *(const f32x4*)(lds_a + i * kTileBytes + lane * 32 + 16 * h);
        q[i] = *(const f32x4*)(lds_a + i * kTileBytes + 2048 + lane * 32 + 16 * h);
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        f32x4 br = *(const f32x4*)(lds_b + j * kTileBytes + lane * 32 + 16 * h);
        f32x4 bi = *(const f32x4*)(lds_b + j * kTileBytes + 2048 + lane * 32 + 16 * h);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
#pragma unroll
          for (int i = 0; i < MB; ++i) {
            gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(p[i][e], br[e], gr[i][j], 0, 0, 0);
            gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(q[i][e], bi[e], gr[i][j], 0, 0, 0);
            gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(p[i][e], bi[e], gi[i][j], 0, 0, 0);
            gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-q[i][e], br[e], gi[i][j], 0, 0, 0);
          }
        }
      }
    }
  } else {
    using half_t = typename std::conditional<PREC == LRS_BF16X2, bf16x8, f16x8>::type;
    half_t ph[MB], pl[MB], qh[MB], ql[MB], nqh[MB], nql[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const unsigned char* a = lds_a + i * kTileBytes + lane * 16;
      ph[i] = *(const half_t*)(a);
      pl[i] = *(const half_t*)(a + 1024);
      qh[i] = *(const half_t*)(a + 2048);
      ql[i] = *(const half_t*)(a + 3072);
      // negation flips the sign bit of every 16-bit element
      u32x4 m = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
      nqh[i] = (half_t)((u32x4)qh[i] ^ m);
      nql[i] = (half_t)((u32x4)ql[i] ^ m);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const unsigned char* b = lds_b + j * kTileBytes + lane * 16;
      half_t rh = *(const half_t*)(b), rl = *(const half_t*)(b + 1024);
      half_t ih = *(const half_t*)(b + 2048), il = *(const half_t*)(b + 3072);
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        if constexpr (PREC == LRS_BF16X2) {
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph[i], rh, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph[i], rl, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pl[i], rh, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qh[i], ih, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(qh[i], il, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ql[i], ih, gr[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph[i], ih, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ph[i], il, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pl[i], ih, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nqh[i], rh, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nqh[i], rl, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nql[i], rh, gi[i][j], 0, 0, 0);
        } else {
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ph[i], rh, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ph[i], rl, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(pl[i], rh, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(qh[i], ih, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(qh[i], il, gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ql[i], ih, gr[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ph[i], ih, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ph[i], il, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(pl[i], ih, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(nqh[i], rh, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(nqh[i], rl, gi[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(nql[i], rh, gi[i][j], 0, 0, 0);
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------- kernel
template <int PREC, int WMW, int WNW, int MB, int NB, int MODE>
__global__ __launch_bounds__(WMW * WNW * 64) void chi0_kernel(Chi0Params P) {
  using acc_t = typename Prec<PREC>::acc_t;
  constexpr int KC = Prec<PREC>::KC;
  constexpr int BM = WMW * MB * 16;
  constexpr int BN = WNW * NB * 16;
  constexpr int THREADS = WMW * WNW * 64;
  constexpr int A_BYTES = (BM / 16) * kTileBytes;
  constexpr int B_BYTES = (BN / 16) * kTileBytes;
  __shared__ __attribute__((aligned(16))) unsigned char lds[A_BYTES + B_BYTES];
  unsigned char* lds_a = lds;
  unsigned char* lds_b = lds + A_BYTES;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WNW, wn = wave % WNW;
  const int G = gridDim.x;
  const int bslot = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int nch = P.nch_o + P.nch_u;

  for (long long tau = bslot; tau < P.ntiles; tau += G) {
    const TileDesc td = P.tiles[tau];
    double chi[MB][NB][4];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) chi[i][j][e] = 0.0;

    for (int t = 0; t < P.T; ++t) {
      acc_t go_r[MB][NB], go_i[MB][NB], gu_r[MB][NB], gu_i[MB][NB];
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          go_r[i][j] = acc_t{0, 0, 0, 0};
          go_i[i][j] = acc_t{0, 0, 0, 0};
          gu_r[i][j] = acc_t{0, 0, 0, 0};
          gu_i[i][j] = acc_t{0, 0, 0, 0};
        }
      for (int ch = 0; ch < nch; ++ch) {
        const int kbase = ch * KC;
        __syncthreads();
        // site operand, weighted by this term
        for (int it = tid; it < BM * 4; it += THREADS)
          stage_a_item<PREC>(P, lds_a, it >> 2, it & 3, td.a_row0 + (it >> 2), t, kbase);
        // column operand: straight copy of BN/16 fragment tiles
        const unsigned char* bsrc =
            P.b + ((size_t)(td.b_col0 >> 4) * P.b_nchunks + ch) * kTileBytes;
        for (int it = tid; it < (BN / 16) * (kTileBytes / 16); it += THREADS) {
          const int blk = it / (kTileBytes / 16), off = it % (kTileBytes / 16);
          *(u32x4*)(lds_b + blk * kTileBytes + off * 16) =
              *(const u32x4*)(bsrc + (size_t)blk * P.b_nchunks * kTileBytes + off * 16);
        }
        __syncthreads();
        const unsigned char* wa = lds_a + wm * MB * kTileBytes;
        const unsigned char* wb = lds_b + wn * NB * kTileBytes;
        if (ch < P.nch_o)
          mma_chunk<PREC, MB, NB>(wa, wb, lane, go_r, go_i);
        else
          mma_chunk<PREC, MB, NB>(wa, wb, lane, gu_r, gu_i);
      }
      if constexpr (MODE == 1) {
        // adjoint: Hu = lam * conj(G_u), Ho = lam * conj(G_o) on this tile (single term)
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int rr = (PREC == LRS_FP64) ? (4 * e + (lane >> 4)) : (4 * (lane >> 4) + e);
              const int row = (wm * MB + i) * 16 + rr;
              const int col = (wn * NB + j) * 16 + (lane & 15);
              if (row < td.nrows && col < td.ncols) {
                const long long o = td.out_off + (long long)row * td.ldo + col;
                const double l = P.lam[o];
                P.hu_re[o] = l * (double)gu_r[i][j][e];
                P.hu_im[o] = -l * (double)gu_i[i][j][e];
                P.ho_re[o] = l * (double)go_r[i][j][e];
                P.ho_im[o] = -l * (double)go_i[i][j][e];
              }
            }
      } else {
        const double ct = P.c[t];
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              chi[i][j][e] += ct * ((double)go_r[i][j][e] * (double)gu_r[i][j][e] +
                                    (double)go_i[i][j][e] * (double)gu_i[i][j][e]);
      }
    }
    if constexpr (MODE == 1) continue;
    // store: f32 16x16 accumulators hold (row 4*(lane/16)+e, col lane%16); the f64 16x16x4
    // accumulator holds (row 4*e + lane/16, col lane%16)
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int rr = (PREC == LRS_FP64) ? (4 * e + (lane >> 4)) : (4 * (lane >> 4) + e);
          const int row = (wm * MB + i) * 16 + rr;
          const int col = (wn * NB + j) * 16 + (lane & 15);
          if (row < td.nrows && col < td.ncols)
            P.out[td.out_off + (long long)row * td.ldo + col] = P.pref * chi[i][j][e];
        }
  }
}

// variant table: {WMW, WNW, MB, NB}
template <int PREC, int V>
struct Variant;
#define LRS_VARIANT(PR, V, A, B, C, D)                                  \
  template <>                                                          \
  struct Variant<PR, V> {                                              \
    static constexpr int WMW = A, WNW = B, MB = C, NB = D;             \
  };
LRS_VARIANT(LRS_FP64, 0, 2, 2, 2, 2)
LRS_VARIANT(LRS_FP64, 1, 2, 2, 2, 1)
LRS_VARIANT(LRS_FP64, 2, 4, 2, 1, 2)
LRS_VARIANT(LRS_FP32, 0, 2, 2, 2, 4)
LRS_VARIANT(LRS_FP32, 1, 2, 2, 2, 2)
LRS_VARIANT(LRS_FP32, 2, 4, 2, 1, 4)
LRS_VARIANT(LRS_BF16X2, 0, 2, 2, 2, 4)
LRS_VARIANT(LRS_BF16X2, 1, 2, 2, 2, 2)
LRS_VARIANT(LRS_BF16X2, 2, 4, 2, 1, 4)
LRS_VARIANT(LRS_FP16X2, 0, 2, 2, 2, 4)
LRS_VARIANT(LRS_FP16X2, 1, 2, 2, 2, 2)
LRS_VARIANT(LRS_FP16X2, 2, 4, 2, 1, 4)
#undef LRS_VARIANT
constexpr int kNumVariants = 3;

template <int PREC, int V>
hipError_t launch_v(int grid, const Chi0Params& P, hipStream_t s) {
  using Vt = Variant<PREC, V>;
  hipLaunchKernelGGL((chi0_kernel<PREC, Vt::WMW, Vt::WNW, Vt::MB, Vt::NB, 0>), dim3(grid),
                     dim3(Vt::WMW * Vt::WNW * 64), 0, s, P);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_p(int variant, int grid, const Chi0Params& P, hipStream_t s) {
  switch (variant) {
    case 0: return launch_v<PREC, 0>(grid, P, s);
    case 1: return launch_v<PREC, 1>(grid, P, s);
    case 2: return launch_v<PREC, 2>(grid, P, s);
  }
  return hipErrorInvalidValue;
}

template <int PREC, int V>
TileShape shape_v() {
  using Vt = Variant<PREC, V>;
  return TileShape{Vt::WMW * Vt::MB * 16, Vt::WNW * Vt::NB * 16, Vt::WMW * Vt::WNW * 64};
}
template <int PREC>
TileShape shape_p(int v) {
  switch (v) {
    case 0: return shape_v<PREC, 0>();
    case 1: return shape_v<PREC, 1>();
    default: return shape_v<PREC, 2>();
  }
}

}  // namespace

int chi0_num_variants(int) { return kNumVariants; }

// fastest variant measured on the precision workload (the tuner can override it)
int chi0_default_variant(int) { return 2; }

namespace {
template <int PREC, int V>
int occ_v() {
  using Vt = Variant<PREC, V>;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, reinterpret_cast<const void*>(&chi0_kernel<PREC, Vt::WMW, Vt::WNW, Vt::MB, Vt::NB, 0>),
          Vt::WMW * Vt::WNW * 64, 0) != hipSuccess)
    return 1;
  return n;
}
template <int PREC>
int occ_p(int v) {
  switch (v) {
    case 0: return occ_v<PREC, 0>();
    case 1: return occ_v<PREC, 1>();
    default: return occ_v<PREC, 2>();
  }
}
}  // namespace

int chi0_blocks_per_cu(int prec, int variant) {
  switch (prec) {
    case LRS_FP64: return occ_p<LRS_FP64>(variant);
    case LRS_FP32: return occ_p<LRS_FP32>(variant);
    case LRS_BF16X2: return occ_p<LRS_BF16X2>(variant);
    default: return occ_p<LRS_FP16X2>(variant);
  }
}

TileShape chi0_shape(int prec, int variant) {
  switch (prec) {
    case LRS_FP64: return shape_p<LRS_FP64>(variant);
    case LRS_FP32: return shape_p<LRS_FP32>(variant);
    case LRS_BF16X2: return shape_p<LRS_BF16X2>(variant);
    default: return shape_p<LRS_FP16X2>(variant);
  }
}

hipError_t launch_chi0(int prec, int variant, int grid, const void* a_re, const void* a_im,
                       int lda, const void* b_tiles, int b_nchunks, const void* w,
                       const double* c, int T, int nch_o, int nch_u, const TileDesc* tiles,
                       int ntiles, double* out, double pref, float a_scale, hipStream_t s) {
  Chi0Params P;
  P.a_re = a_re;
  P.a_im = a_im;
  P.lda = lda;
  P.b = (const unsigned char*)b_tiles;
  P.b_nchunks = b_nchunks;
  P.w = w;
  P.c = c;
  P.T = T;
  P.nch_o = nch_o;
  P.nch_u = nch_u;
  P.tiles = tiles;
  P.ntiles = ntiles;
  P.out = out;
  P.pref = pref;
  P.a_scale = a_scale;
  P.lam = nullptr;
  P.hu_re = P.hu_im = P.ho_re = P.ho_im = nullptr;
  switch (prec) {
    case LRS_FP64: return launch_p<LRS_FP64>(variant, grid, P, s);
    case LRS_FP32: return launch_p<LRS_FP32>(variant, grid, P, s);
    case LRS_BF16X2: return launch_p<LRS_BF16X2>(variant, grid, P, s);
    case LRS_FP16X2: return launch_p<LRS_FP16X2>(variant, grid, P, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_green_adjoint(int grid, const void* a_re, const void* a_im, int lda,
                                const void* b_tiles, int b_nchunks, const double* w,
                                const double* c, int nch_o, int nch_u, const TileDesc* tiles,
                                int ntiles, const double* lam, double* hu_re, double* hu_im,
                                double* ho_re, double* ho_im, hipStream_t s) {
  Chi0Params P;
  P.a_re = a_re;
  P.a_im = a_im;
  P.lda = lda;
  P.b = (const unsigned char*)b_tiles;
  P.b_nchunks = b_nchunks;
  P.w = w;
  P.c = c;
  P.T = 1;
  P.nch_o = nch_o;
  P.nch_u = nch_u;
  P.tiles = tiles;
  P.ntiles = ntiles;
  P.out = nullptr;
  P.pref = 1.0;
  P.a_scale = 1.f;
  P.lam = lam;
  P.hu_re = hu_re;
  P.hu_im = hu_im;
  P.ho_re = ho_re;
  P.ho_im = ho_im;
  using Vt = Variant<LRS_FP64, 0>;
  hipLaunchKernelGGL((chi0_kernel<LRS_FP64, Vt::WMW, Vt::WNW, Vt::MB, Vt::NB, 1>), dim3(grid),
                     dim3(Vt::WMW * Vt::WNW * 64), 0, s, P);
  return hipGetLastError();
}

}  // namespace lrs
