// chi0 on the matrix cores (Sec. VI.D with the energy quadrature of Appendix D.1.b).
//
// For one output tile (rows r of the site operand x columns r' of the column operand) and
// each quadrature term l, a workgroup forms the two weighted Green's function tiles
//     G_o^l(r,r') = sum_{K occ}   conj(psi_K(r)) alpha_l(K) psi_K(r')
//     G_u^l(r,r') = sum_{K unocc} conj(psi_K(r)) beta_l(K)  psi_K(r')
// as complex GEMMs in the real 4M form (G_r = p b_r + q b_i, G_i = p b_i - q b_r with
// p + i q = weight * psi(r)) on MFMA, then accumulates
//     chi(r,r') += c_l (Re G_o Re G_u + Im G_o Im G_u)
// in FP64 (read-modify-write of the tile's own output entries once per term).  The last
// term applies the prefactor -2 s / N_k^2.
//
// Operands.  Both sides arrive as 4 KiB fragment tiles (16 rows or columns x one K chunk,
// every lane's matrix-core operand contiguous): the column operand is packed once per set of
// orbitals; the weighted site operand of every term is built once per call by
// prep_site_kernel (the per-term weight lives on the small site side, so the large column
// operand is the same for every term).  BF16X2 / FP16X2 carry hi + lo halves of each value;
// each real product takes hi*hi + hi*lo + lo*hi (lo*lo dropped) with FP32 accumulation.
//
// Pipeline.  The chunks of a tile (term-major, then K) stream through a two-slot LDS ring
// filled by 16-byte direct-to-LDS loads, with two register sets of operand fragments: while
// the matrix cores work on chunk q, chunk q+1's fragments are read from LDS and chunk q+2's
// tiles travel from global memory into the slot chunk q came from (see chi0_kernel).
//
// Persistent launch: gridDim.x workgroups walk a host-built tile list; workgroup b handles
// tiles b' + i * gridDim.x with b' = (b % 8) * (gridDim.x / 8) + b / 8, so that the
// workgroups resident on one XCD (dispatch is round-robin over the 8 XCDs) take a contiguous
// run of the list, which the host orders in 8 x 8 groups of (row tile, column tile): the
// concurrently running workgroups of an XCD share operand tiles in that XCD's L2.
#include <hip/hip_runtime.h>

#include "lrs_internal.h"
#include "ring.h"

namespace lrs {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned int)))) unsigned int u32x4;
typedef __attribute__((__vector_size__(2 * sizeof(unsigned int)))) unsigned int u32x2;
typedef int i32x8 __attribute__((ext_vector_type(8)));   // 32 fp8 values

struct Chi0Params {
  const unsigned char* a;       // weighted site operand tiles [term][chunk][rowblock][tile]
  int a_nrb;                    // row blocks per term in a
  const unsigned char* b;       // column operand tiles [chunk][colblock][tile]
  int b_ncb;                    // column blocks in b
  int nch;                      // chunks per term (= K_pad / chunk)
  const double* c;              // [T]
  const double* ci;             // [T] imaginary parts of the term coefficients, or null
  int T, nch_o;
  const TileDesc* tiles;
  int ntiles;
  double* out;
  double pref;
  int sym;                      // site blocks from their upper triangle (mode 0)
  unsigned int* sync;           // per-XCD term counters (stride 16), zero at launch; or null
  unsigned char* park;          // per-workgroup space for G_o between the two phases
  // adjoint modes: with T = 1, write lam * conj(G_u) and lam * conj(G_o), as FP64 planes with
  // the block's row stride (mode 1) or as bfloat16 hi/lo in operand tiles (mode 2,
  // h_tile_offset).  With lam_a (complex term coefficients, chi0 at imaginary frequency) the
  // coefficient matrices are Hermitian: adj_c lam + i adj_s lam_a for G_u and
  // adj_c lam - i adj_s lam_a for G_o (lam symmetric, lam_a antisymmetric).
  const double* lam;
  const double* lam_a;
  double adj_c, adj_s;
  double* hu_re;
  double* hu_im;
  double* ho_re;
  double* ho_im;
  __bf16* hs_u;
  __bf16* hs_o;
  // mode 0 on site blocks: keep each term's G_o and G_u (complex: FP64 for the FP64 path, else
  // FP32; the output's element offsets, term stride keep_stride) on and above the diagonal for
  // the adjoint, or null
  void* keep_o;
  void* keep_u;
  long long keep_stride;
};

// x = hi + lo in bfloat16 (hi rounded from x, lo from the remainder), re and im of one
// element into four planes
__device__ __forceinline__ void put_split(__bf16* base, long long plane, long long o, double re,
                                          double im) {
  const __bf16 rh = (__bf16)(float)re, ih = (__bf16)(float)im;
  base[o] = rh;
  base[plane + o] = (__bf16)(float)(re - (double)(float)rh);
  base[2 * plane + o] = ih;
  base[3 * plane + o] = (__bf16)(float)(im - (double)(float)ih);
}

// Matrix-core shape per precision.  FP64 and FP32 use 16 x 16 accumulator blocks (4 values
// per lane); the split 16-bit paths use the 32 x 32 x 16 instructions (16 values per lane),
// which sustain twice the rate of the 16 x 16 x 32 form on gfx950.
//   KC  K values per chunk, TB bytes per fragment tile (16 rows x KC x planes).
template <int PREC>
struct Prec;
template <>
struct Prec<LRS_FP64> {
  using acc_t = f64x4;
  static constexpr int KC = 16, TB = 4096, BLK = 16, ELEMS = 4;
};
// three planes per operand tile: p, q, p - q (rows); b_r, b_i, b_r + b_i (columns)
template <>
struct Prec<LRS_FP64_3M> {
  using acc_t = f64x4;
  static constexpr int KC = 16, TB = 6144, BLK = 16, ELEMS = 4;
};
template <>
struct Prec<LRS_FP32> {
  using acc_t = f32x4;
  static constexpr int KC = 32, TB = 4096, BLK = 16, ELEMS = 4;
};
template <>
struct Prec<LRS_BF16X2> {
  using acc_t = f32x16;
  static constexpr int KC = 16, TB = 2048, BLK = 32, ELEMS = 16;
};
template <>
struct Prec<LRS_FP16X2> {
  using acc_t = f32x16;
  static constexpr int KC = 16, TB = 2048, BLK = 32, ELEMS = 16;
};
// fp16 hi products on v_mfma_f32_32x32x16_f16, the cross terms on
// v_mfma_scale_f32_32x32x64_f8f6f4 (fp8 e4m3, one scale per row and 32-K block); 16 K per chunk
template <>
struct Prec<LRS_F16F8> {
  using acc_t = f32x16;
  static constexpr int KC = 16, TB = 2048, BLK = 32, ELEMS = 16;
};

// Row and column (inside a BLK x BLK accumulator block) of element e of a lane:
//   f32 16x16:   (4 (lane/16) + e, lane%16)
//   f64 16x16x4: (4 e + lane/16, lane%16)
//   f32 32x32:   (8 (e/4) + 4 (lane/32) + e%4, lane%32)
template <int PREC>
__device__ __forceinline__ void elem_rc(int lane, int e, int& r, int& c) {
  if constexpr (PREC == LRS_FP64 || PREC == LRS_FP64_3M) {
    r = 4 * e + (lane >> 4);
    c = lane & 15;
  } else if constexpr (PREC == LRS_FP32) {
    r = 4 * (lane >> 4) + e;
    c = lane & 15;
  } else {
    r = 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    c = lane & 31;
  }
}

template <class T>
__device__ __forceinline__ T zero_acc() {
  T v;
#pragma unroll
  for (int e = 0; e < (int)(sizeof(T) / sizeof(v[0])); ++e) v[e] = 0;
  return v;
}

// ----------------------------------------------------------------------------- site prep
// Weighted site operand for terms [t0, t0 + nt) and row blocks [rb0, rb0 + nrb) of the slot
// layout, with p + i q = w_t(k) * psi_k(row) * a_scale.  One thread per (row block, chunk,
// lane slot) reads that slot's orbital values once and writes the slot of every plane for
// each term in turn:
//   FP64 (chunk 16, 64 slots):  slot l holds row l%16, k = 4 s + l/16, s = 0..3, planes p, q
//                               (FP64 3M: a third plane p - q)
//   FP32 (chunk 32, 64 slots):  slot l holds row l%16, k = 4 s + l/16, s = 0..7, planes p, q
//   split (chunk 16, 32 slots): slot l holds row l%16, k = 8 (l/16) + e, e = 0..7,
//                               planes p_hi, p_lo, q_hi, q_lo
// (a_scale is a power of two, so the product does not depend on the order of the factors)
__device__ inline size_t site_pos(int r, int k, int K_pad) {
  int ch = k >> 4, kl = k & 15;
  return (size_t)r * K_pad + ch * 16 + (kl & 3) * 4 + (kl >> 2);
}

// F16F8 (chunk 16, 32 slots): slot s holds row s%16 and K 8 (s/16) + j, j = 0..7, of the
// chunk: the fp16 hi slot s of planes re and im, and bytes 8 (s/16) .. + 7 of row s%16 of the
// fp8 planes, part 0 = hi * 2^7 and part 1 = lo * 2^18 (the row side's order).
__global__ void prep_site_f16f8_kernel(const double* site, int rows_pad, int K_pad,
                                       const int* slot_row, int rb0, int nrb, const double* w,
                                       int w_stride, int q_woff, int t0, int nt, double a_scale,
                                       unsigned char* out) {
  constexpr int TB = 2048;
  const int nch = K_pad / 16;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)nrb * nch * 32) return;
  const int s = (int)(gid % 32);
  const long long tile = gid / 32;
  const int rb = (int)(tile % nrb);
  const int ch = (int)(tile / nrb);
  const int r = s & 15, h = s >> 4;
  const int row = slot_row[(rb0 + rb) * 16 + r];
  const size_t plane = (size_t)rows_pad * K_pad;
  const int k0 = ch * 16 + 8 * h;
  double p0[8], q0[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (row < 0) {
      p0[j] = 0.0;
      q0[j] = 0.0;
    } else {
      const size_t o = site_pos(row, k0 + j, K_pad);
      p0[j] = site[o] * a_scale;
      q0[j] = site[plane + o] * a_scale;
    }
  }
  for (int t = 0; t < nt; ++t) {
    const double* wt = w + (size_t)(t0 + t) * w_stride + k0;
    unsigned char* base = out + (((size_t)t * nch + ch) * nrb + rb) * TB;
    f16x8 hp, hq;
    unsigned int f8[4][2] = {};     // [re p0, re p1, im p0, im p1][dword]
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float xp = (float)(p0[j] * wt[j]), xq = (float)(q0[j] * wt[q_woff + j]);
      const _Float16 a = (_Float16)xp, b = (_Float16)xq;
      hp[j] = a;
      hq[j] = b;
      const int sh = 8 * (j & 3), dw = j >> 2;
      f8[0][dw] |= e4m3_rn(ldexpf((float)a, kF8HiShift)) << sh;
      f8[1][dw] |= e4m3_rn(ldexpf(xp - (float)a, kF8LoShift)) << sh;
      f8[2][dw] |= e4m3_rn(ldexpf((float)b, kF8HiShift)) << sh;
      f8[3][dw] |= e4m3_rn(ldexpf(xq - (float)b, kF8LoShift)) << sh;
    }
    *(f16x8*)(base + s * 16) = hp;
    *(f16x8*)(base + 512 + s * 16) = hq;
#pragma unroll
    for (int part = 0; part < 4; ++part) {
      u32x2 v = {f8[part][0], f8[part][1]};
      *(u32x2*)(base + 1024 + part * 256 + r * 16 + 8 * h) = v;
    }
  }
}

template <int PREC>
__global__ void prep_site_kernel(const double* site, int rows_pad, int K_pad, const int* slot_row,
                                 int rb0, int nrb, const double* w, int w_stride, int q_woff,
                                 int t0, int nt, double a_scale, unsigned char* out) {
  constexpr int KC = Prec<PREC>::KC, TB = Prec<PREC>::TB;
  constexpr bool SPLIT = PREC == LRS_BF16X2 || PREC == LRS_FP16X2;
  constexpr int SLOTS = SPLIT ? 32 : 64;
  constexpr bool F64 = PREC == LRS_FP64 || PREC == LRS_FP64_3M;
  constexpr int NV = F64 ? 4 : 8;     // values of the slot per plane
  const int nch = K_pad / KC;
  long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long long)nrb * nch * SLOTS) return;
  const int lane = (int)(gid % SLOTS);
  const long long tile = gid / SLOTS;        // ch * nrb + rb
  const int rb = (int)(tile % nrb);
  const int ch = (int)(tile / nrb);
  const int row = slot_row[(rb0 + rb) * 16 + (lane & 15)];
  const size_t plane = (size_t)rows_pad * K_pad;
  int kv[NV];
  double p0[NV], q0[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    kv[v] = SPLIT ? ch * 16 + 8 * (lane >> 4) + v : ch * KC + 4 * v + (lane >> 4);
    if (row < 0) {
      p0[v] = 0.0;
      q0[v] = 0.0;
    } else {
      const size_t o = site_pos(row, kv[v], K_pad);
      p0[v] = site[o] * a_scale;
      q0[v] = site[plane + o] * a_scale;
    }
  }
  for (int t = 0; t < nt; ++t) {
    const double* wt = w + (size_t)(t0 + t) * w_stride;
    const double* wq = wt + q_woff;
    unsigned char* base = out + (((size_t)t * nch + ch) * nrb + rb) * TB;
    if constexpr (F64) {
      f64x4 vp, vq;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        vp[v] = p0[v] * wt[kv[v]];
        vq[v] = q0[v] * wq[kv[v]];
      }
      f64x4* d = (f64x4*)base;
      d[lane] = vp;
      d[64 + lane] = vq;
      if constexpr (PREC == LRS_FP64_3M) d[128 + lane] = vp - vq;
    } else if constexpr (PREC == LRS_FP32) {
      float* d = (float*)base;
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        d[lane * 8 + v] = (float)(p0[v] * wt[kv[v]]);
        d[512 + lane * 8 + v] = (float)(q0[v] * wq[kv[v]]);
      }
    } else {
      using elem_t = typename std::conditional<PREC == LRS_BF16X2, __bf16, _Float16>::type;
      using vec_t = typename std::conditional<PREC == LRS_BF16X2, bf16x8, f16x8>::type;
      // the slot's 8 values of each plane are 16 contiguous bytes: one store per plane
      vec_t vph, vpl, vqh, vql;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double p = p0[e] * wt[kv[e]], q = q0[e] * wq[kv[e]];
        const elem_t ph = (elem_t)(float)p, qh = (elem_t)(float)q;
        vph[e] = ph;
        vpl[e] = (elem_t)(float)(p - (double)(float)ph);
        vqh[e] = qh;
        vql[e] = (elem_t)(float)(q - (double)(float)qh);
      }
      vec_t* d = (vec_t*)base;
      d[lane] = vph;
      d[32 + lane] = vpl;
      d[64 + lane] = vqh;
      d[96 + lane] = vql;
    }
  }
}

// ----------------------------------------------------------------------------- MFMA step
// One chunk of the wave's MB x NB tiles of 16 rows, in two parts: load_frags() reads every
// operand fragment the chunk needs from LDS into registers, mma_frags() runs the matrix-core
// instructions on them.
template <int PREC, int MB, int NB>
struct Frags;

template <int MB, int NB>
struct Frags<LRS_FP64, MB, NB> {
  f64x4 p[MB], q[MB], br[NB], bi[NB];   // element s <-> k = 4 s + lane/16
};
template <int MB, int NB>
struct Frags<LRS_FP64_3M, MB, NB> {
  f64x4 p[MB], q[MB], d[MB], br[NB], bi[NB], bs[NB];
};
template <int MB, int NB>
struct Frags<LRS_FP32, MB, NB> {
  f32x4 p[MB][2], q[MB][2], br[NB][2], bi[NB][2];   // [h][e] <-> k = 4 (4 h + e) + lane/16
};
// split paths: one 32-row block per two 16-row tiles; lane l reads row l%32 of the block at
// k = 8 (l/32) + e, which sits in tile (l%32)/16 at slot (l/32) * 16 + l%16.
template <int MB, int NB>
struct Frags<LRS_BF16X2, MB, NB> {
  bf16x8 ph[MB / 2], pl[MB / 2], qh[MB / 2], ql[MB / 2];
  bf16x8 rh[NB / 2], rl[NB / 2], ih[NB / 2], il[NB / 2];
};
template <int MB, int NB>
struct Frags<LRS_FP16X2, MB, NB> {
  f16x8 ph[MB / 2], pl[MB / 2], qh[MB / 2], ql[MB / 2];
  f16x8 rh[NB / 2], rl[NB / 2], ih[NB / 2], il[NB / 2];
};
// F16F8: per 32-row block the fp16 hi values of the chunk (lane l: row l%32, K 8 (l/32) + e)
// and a 32-byte fp8 fragment (lane l: row l%32, parts 0 and 1 of re in lanes 0-31, of im in
// lanes 32-63).  The column side has a second fp8 fragment with the components the other way
// round (im in lanes 0-31, re in 32-63), which the imaginary part's cross terms take: reading
// it from LDS again costs less than exchanging the lane halves in registers.
template <int MB, int NB>
struct Frags<LRS_F16F8, MB, NB> {
  f16x8 p[MB / 2], q[MB / 2];
  i32x8 a8[MB / 2];
  f16x8 r[NB / 2], i[NB / 2];
  i32x8 br8[NB / 2], bi8[NB / 2];
};

// fp8 fragment of 32 bytes from two 16-byte parts 256 bytes apart
__device__ __forceinline__ i32x8 load_f8(const unsigned char* p) {
  const u32x4 a = *(const u32x4*)p, b = *(const u32x4*)(p + 256);
  i32x8 v;
  v[0] = (int)a[0]; v[1] = (int)a[1]; v[2] = (int)a[2]; v[3] = (int)a[3];
  v[4] = (int)b[0]; v[5] = (int)b[1]; v[6] = (int)b[2]; v[7] = (int)b[3];
  return v;
}

template <int PREC, int MB, int NB, bool RE = false>
__device__ __forceinline__ void load_frags(const unsigned char* lds_a, const unsigned char* lds_b,
                                           int lane, Frags<PREC, MB, NB>& f) {
  constexpr int TB = Prec<PREC>::TB;
  if constexpr (PREC == LRS_FP64) {
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      f.p[i] = *(const f64x4*)(lds_a + i * TB + lane * 32);
      f.q[i] = *(const f64x4*)(lds_a + i * TB + 2048 + lane * 32);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      f.br[j] = *(const f64x4*)(lds_b + j * TB + lane * 32);
      f.bi[j] = *(const f64x4*)(lds_b + j * TB + 2048 + lane * 32);
    }
  } else if constexpr (PREC == LRS_FP64_3M) {
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      f.p[i] = *(const f64x4*)(lds_a + i * TB + lane * 32);
      f.q[i] = *(const f64x4*)(lds_a + i * TB + 2048 + lane * 32);
      f.d[i] = *(const f64x4*)(lds_a + i * TB + 4096 + lane * 32);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      f.br[j] = *(const f64x4*)(lds_b + j * TB + lane * 32);
      f.bi[j] = *(const f64x4*)(lds_b + j * TB + 2048 + lane * 32);
      f.bs[j] = *(const f64x4*)(lds_b + j * TB + 4096 + lane * 32);
    }
  } else if constexpr (PREC == LRS_FP32) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        f.p[i][h] = *(const f32x4*)(lds_a + i * TB + lane * 32 + 16 * h);
        f.q[i][h] = *(const f32x4*)(lds_a + i * TB + 2048 + lane * 32 + 16 * h);
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        f.br[j][h] = *(const f32x4*)(lds_b + j * TB + lane * 32 + 16 * h);
        f.bi[j][h] = *(const f32x4*)(lds_b + j * TB + 2048 + lane * 32 + 16 * h);
      }
    }
  } else if constexpr (PREC == LRS_F16F8) {
    // a 32-row block is two 2 KiB tiles; lane l reads fp16 slot (l/32) * 16 + l%16 of tile
    // (l%32)/16 and row l%16 of that tile's fp8 planes of component l/32 (own) or the other
    const int tofs = ((lane & 31) >> 4) * TB + (lane & 15) * 16;
    const int lofs = tofs + (lane >> 5) * 256;
    const int own = tofs + 1024 + (lane >> 5) * 512, other = tofs + 1024 + (1 - (lane >> 5)) * 512;
#pragma unroll
    for (int i = 0; i < MB / 2; ++i) {
      const unsigned char* a = lds_a + i * 2 * TB;
      f.p[i] = *(const f16x8*)(a + lofs);
      f.q[i] = *(const f16x8*)(a + lofs + 512);
      f.a8[i] = load_f8(a + own);
    }
#pragma unroll
    for (int j = 0; j < NB / 2; ++j) {
      const unsigned char* b = lds_b + j * 2 * TB;
      f.r[j] = *(const f16x8*)(b + lofs);
      f.i[j] = *(const f16x8*)(b + lofs + 512);
      f.br8[j] = load_f8(b + own);
      if constexpr (!RE) f.bi8[j] = load_f8(b + other);
    }
  } else {
    using half_t = typename std::conditional<PREC == LRS_BF16X2, bf16x8, f16x8>::type;
    const int lofs = ((lane & 31) >> 4) * TB + (lane >> 5) * 256 + (lane & 15) * 16;
#pragma unroll
    for (int i = 0; i < MB / 2; ++i) {
      const unsigned char* a = lds_a + i * 2 * TB + lofs;
      f.ph[i] = *(const half_t*)(a);
      f.pl[i] = *(const half_t*)(a + 512);
      f.qh[i] = *(const half_t*)(a + 1024);
      f.ql[i] = *(const half_t*)(a + 1536);
    }
#pragma unroll
    for (int j = 0; j < NB / 2; ++j) {
      const unsigned char* b = lds_b + j * 2 * TB + lofs;
      f.rh[j] = *(const half_t*)(b);
      f.rl[j] = *(const half_t*)(b + 512);
      f.ih[j] = *(const half_t*)(b + 1024);
      f.il[j] = *(const half_t*)(b + 1536);
    }
  }
}

template <int PREC, int MB, int NB>
__device__ __forceinline__ void mma_frags(
    const Frags<PREC, MB, NB>& f,
    typename Prec<PREC>::acc_t (&gr)[MB * 16 / Prec<PREC>::BLK][NB * 16 / Prec<PREC>::BLK],
    typename Prec<PREC>::acc_t (&gi)[MB * 16 / Prec<PREC>::BLK][NB * 16 / Prec<PREC>::BLK]) {
  if constexpr (PREC == LRS_FP64) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          gr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.p[i][s], f.br[j][s], gr[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.p[i][s], f.bi[j][s], gi[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.q[i][s], f.bi[j][s], gr[i][j], 0, 0, 0);
          gi[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-f.q[i][s], f.br[j][s], gi[i][j], 0, 0, 0);
        }
  } else if constexpr (PREC == LRS_FP32) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            const float p = f.p[i][h][e], q = f.q[i][h][e];
            const float br = f.br[j][h][e], bi = f.bi[j][h][e];
            gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(p, br, gr[i][j], 0, 0, 0);
            gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(p, bi, gi[i][j], 0, 0, 0);
            gr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(q, bi, gr[i][j], 0, 0, 0);
            gi[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(-q, br, gi[i][j], 0, 0, 0);
          }
  } else if constexpr (PREC == LRS_F16F8) {
    // hi * hi on the fp16 instruction; hi * lo and lo * hi of both real products of a complex
    // multiply-add on one scaled fp8 instruction: its K runs over (re, im) x (block 0, block 1)
    // with block 0 = row hi x column lo (scales 2^-7, 2^-18) and block 1 = row lo x column hi
    // (2^-18, 2^-7).  The row fragment carries p (lanes 0-31) and q (lanes 32-63), the column
    // fragment b_r and b_i for G_r, or b_i and -b_r for G_i.  Each stage updates every block
    // of one accumulator array before the next, so dependent instructions are far apart.
    const int lane = __lane_id();
    const int sa = lane < 32 ? 127 - kF8HiShift : 127 - kF8LoShift;
    const int sb = lane < 32 ? 127 - kF8LoShift : 127 - kF8HiShift;
    const u32x4 m16 = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    const int m8 = lane < 32 ? 0 : (int)0x80808080u;
    auto h = [](f16x8 a, f16x8 b, f32x16 c) {
      return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    };
    auto e = [&](i32x8 a, i32x8 b, f32x16 c) {
      return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
    };
    f16x8 nq[MB / 2];
    i32x8 bi8[NB / 2];
#pragma unroll
    for (int i = 0; i < MB / 2; ++i) nq[i] = (f16x8)((u32x4)f.q[i] ^ m16);
#pragma unroll
    for (int j = 0; j < NB / 2; ++j) bi8[j] = f.bi8[j] ^ m8;
#define LRS_F16F8_STAGE(ACC, OP, A, B)         \
  _Pragma("unroll") for (int i = 0; i < MB / 2; ++i) \
    _Pragma("unroll") for (int j = 0; j < NB / 2; ++j) ACC[i][j] = OP(A[i], B[j], ACC[i][j]);
    // G_r += p b_r + q b_i,  G_i += p b_i - q b_r
    LRS_F16F8_STAGE(gr, h, f.p, f.r)
    LRS_F16F8_STAGE(gi, h, f.p, f.i)
    LRS_F16F8_STAGE(gr, e, f.a8, f.br8)
    LRS_F16F8_STAGE(gi, e, f.a8, bi8)
    LRS_F16F8_STAGE(gr, h, f.q, f.i)
    LRS_F16F8_STAGE(gi, h, nq, f.r)
#undef LRS_F16F8_STAGE
  } else {
    using half_t = typename std::conditional<PREC == LRS_BF16X2, bf16x8, f16x8>::type;
    // negation flips the sign bit of every 16-bit element
    const u32x4 m = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    auto mf = [](half_t a, half_t b, f32x16 c) {
      if constexpr (PREC == LRS_BF16X2)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
      else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    };
#pragma unroll
    for (int i = 0; i < MB / 2; ++i) {
      const half_t ph = f.ph[i], pl = f.pl[i], qh = f.qh[i], ql = f.ql[i];
      const half_t nqh = (half_t)((u32x4)qh ^ m);
      const half_t nql = (half_t)((u32x4)ql ^ m);
      // G_r += p b_r + q b_i, G_i += p b_i - q b_r; consecutive instructions update
      // different accumulators
#pragma unroll
      for (int j = 0; j < NB / 2; ++j) {
        gr[i][j] = mf(ph, f.rh[j], gr[i][j]);
        gi[i][j] = mf(ph, f.ih[j], gi[i][j]);
      }
#pragma unroll
      for (int j = 0; j < NB / 2; ++j) {
        gr[i][j] = mf(ph, f.rl[j], gr[i][j]);
        gi[i][j] = mf(ph, f.il[j], gi[i][j]);
      }
#pragma unroll
      for (int j = 0; j < NB / 2; ++j) {
        gr[i][j] = mf(pl, f.rh[j], gr[i][j]);
        gi[i][j] = mf(pl, f.ih[j], gi[i][j]);
      }
#pragma unroll
      for (int j = 0; j < NB / 2; ++j) {
        gr[i][j] = mf(qh, f.ih[j], gr[i][j]);
        gi[i][j] = mf(nqh, f.rh[j], gi[i][j]);
      }
#pragma unroll
      for (int j = 0; j < NB / 2; ++j) {
        gr[i][j] = mf(qh, f.il[j], gr[i][j]);
        gi[i][j] = mf(nqh, f.rl[j], gi[i][j]);
      }
#pragma unroll
      for (int j = 0; j < NB / 2; ++j) {
        gr[i][j] = mf(ql, f.ih[j], gr[i][j]);
        gi[i][j] = mf(nql, f.rh[j], gi[i][j]);
      }
    }
  }
}

// Real orbitals (kernel mode 3): each operand slot carries two real orbitals, the first in the
// "re" plane and the second in the "im" plane (two K values per slot), so G = sum over both
// planes of p b, which is the real-part update of the complex product; G_i stays zero.
template <int PREC, int MB, int NB>
__device__ __forceinline__ void mma_frags_re(
    const Frags<PREC, MB, NB>& f,
    typename Prec<PREC>::acc_t (&gr)[MB * 16 / Prec<PREC>::BLK][NB * 16 / Prec<PREC>::BLK]) {
  static_assert(PREC == LRS_FP64 || PREC == LRS_F16F8, "real orbitals: FP64 and F16F8");
  if constexpr (PREC == LRS_FP64) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          gr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.p[i][s], f.br[j][s], gr[i][j], 0, 0, 0);
          gr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.q[i][s], f.bi[j][s], gr[i][j], 0, 0, 0);
        }
  } else {
    const int lane = __lane_id();
    const int sa = lane < 32 ? 127 - kF8HiShift : 127 - kF8LoShift;
    const int sb = lane < 32 ? 127 - kF8LoShift : 127 - kF8HiShift;
#pragma unroll
    for (int i = 0; i < MB / 2; ++i)
#pragma unroll
      for (int j = 0; j < NB / 2; ++j)
        gr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(f.p[i], f.r[j], gr[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < MB / 2; ++i)
#pragma unroll
      for (int j = 0; j < NB / 2; ++j)
        gr[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(f.a8[i], f.br8[j], gr[i][j], 0,
                                                                  0, 0, sa, 0, sb);
#pragma unroll
    for (int i = 0; i < MB / 2; ++i)
#pragma unroll
      for (int j = 0; j < NB / 2; ++j)
        gr[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(f.q[i], f.i[j], gr[i][j], 0, 0, 0);
  }
}

// FP64 3M: T1 = p b_r into gr, T2 = q b_i into gi, T3 = (p - q)(b_r + b_i) into gx, per
// k-step of the chunk; combine_3m turns them into G_r = T1 + T2 and G_i = T3 - T1 + T2.
template <int MB, int NB>
__device__ __forceinline__ void mma_frags_3m(const Frags<LRS_FP64_3M, MB, NB>& f,
                                             f64x4 (&gr)[MB][NB], f64x4 (&gi)[MB][NB],
                                             f64x4 (&gx)[MB][NB]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        gr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.p[i][s], f.br[j][s], gr[i][j], 0, 0, 0);
        gi[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.q[i][s], f.bi[j][s], gi[i][j], 0, 0, 0);
        gx[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.d[i][s], f.bs[j][s], gx[i][j], 0, 0, 0);
      }
}
template <int MB, int NB>
__device__ __forceinline__ void combine_3m(f64x4 (&gr)[MB][NB], f64x4 (&gi)[MB][NB],
                                           const f64x4 (&gx)[MB][NB]) {
#pragma unroll
  for (int i = 0; i < MB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const f64x4 t2 = gi[i][j];
      gi[i][j] = gx[i][j] - gr[i][j] + t2;
      gr[i][j] = gr[i][j] + t2;
    }
}

// Split paths with rotating B fragments: the A fragments of a chunk are double-buffered, the B
// fragments are single-buffered and refilled block column by block column: once the matrix-core
// instructions of B block j have issued, block j is read again from the next chunk's slot.  This
// keeps a 64 x 128 wave tile (256 accumulator registers) within the register file.
template <int PREC, int MB>
struct FragsA {
  using half_t = typename std::conditional<PREC == LRS_BF16X2, bf16x8, f16x8>::type;
  half_t ph[MB / 2], pl[MB / 2], qh[MB / 2], ql[MB / 2];
};
template <int PREC, int NB>
struct FragsB {
  using half_t = typename std::conditional<PREC == LRS_BF16X2, bf16x8, f16x8>::type;
  half_t rh[NB / 2], rl[NB / 2], ih[NB / 2], il[NB / 2];
};

__device__ __forceinline__ int split_lane_ofs(int lane, int tb) {
  return ((lane & 31) >> 4) * tb + (lane >> 5) * 256 + (lane & 15) * 16;
}

template <int PREC, int MB>
__device__ __forceinline__ void load_a_split(const unsigned char* lds_a, int lane,
                                             FragsA<PREC, MB>& f) {
  using half_t = typename FragsA<PREC, MB>::half_t;
  constexpr int TB = Prec<PREC>::TB;
  const int lofs = split_lane_ofs(lane, TB);
#pragma unroll
  for (int i = 0; i < MB / 2; ++i) {
    const unsigned char* a = lds_a + i * 2 * TB + lofs;
    f.ph[i] = *(const half_t*)(a);
    f.pl[i] = *(const half_t*)(a + 512);
    f.qh[i] = *(const half_t*)(a + 1024);
    f.ql[i] = *(const half_t*)(a + 1536);
  }
}

template <int PREC, int NB>
__device__ __forceinline__ void load_b_split(const unsigned char* lds_b, int lane, int j,
                                             FragsB<PREC, NB>& f) {
  using half_t = typename FragsB<PREC, NB>::half_t;
  constexpr int TB = Prec<PREC>::TB;
  const unsigned char* b = lds_b + j * 2 * TB + split_lane_ofs(lane, TB);
  f.rh[j] = *(const half_t*)(b);
  f.rl[j] = *(const half_t*)(b + 512);
  f.ih[j] = *(const half_t*)(b + 1024);
  f.il[j] = *(const half_t*)(b + 1536);
}

// the matrix-core instructions of B block column j: per product, the A blocks in turn, G_r
// and G_i alternating, so that consecutive instructions update different accumulators
template <int PREC, int MB, int NB>
__device__ __forceinline__ void mma_col_split(const FragsA<PREC, MB>& a, const FragsB<PREC, NB>& b,
                                              int j, f32x16 (&gr)[MB / 2][NB / 2],
                                              f32x16 (&gi)[MB / 2][NB / 2]) {
  using half_t = typename FragsA<PREC, MB>::half_t;
  const u32x4 m = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  auto mf = [](half_t x, half_t y, f32x16 c) {
    if constexpr (PREC == LRS_BF16X2)
      return __builtin_amdgcn_mfma_f32_32x32x16_bf16(x, y, c, 0, 0, 0);
    else
      return __builtin_amdgcn_mfma_f32_32x32x16_f16(x, y, c, 0, 0, 0);
  };
  half_t nqh[MB / 2], nql[MB / 2];
#pragma unroll
  for (int i = 0; i < MB / 2; ++i) {
    nqh[i] = (half_t)((u32x4)a.qh[i] ^ m);
    nql[i] = (half_t)((u32x4)a.ql[i] ^ m);
  }
#pragma unroll
  for (int i = 0; i < MB / 2; ++i) {
    gr[i][j] = mf(a.ph[i], b.rh[j], gr[i][j]);
    gi[i][j] = mf(a.ph[i], b.ih[j], gi[i][j]);
  }
#pragma unroll
  for (int i = 0; i < MB / 2; ++i) {
    gr[i][j] = mf(a.ph[i], b.rl[j], gr[i][j]);
    gi[i][j] = mf(a.ph[i], b.il[j], gi[i][j]);
  }
#pragma unroll
  for (int i = 0; i < MB / 2; ++i) {
    gr[i][j] = mf(a.pl[i], b.rh[j], gr[i][j]);
    gi[i][j] = mf(a.pl[i], b.ih[j], gi[i][j]);
  }
#pragma unroll
  for (int i = 0; i < MB / 2; ++i) {
    gr[i][j] = mf(a.qh[i], b.ih[j], gr[i][j]);
    gi[i][j] = mf(nqh[i], b.rh[j], gi[i][j]);
  }
#pragma unroll
  for (int i = 0; i < MB / 2; ++i) {
    gr[i][j] = mf(a.qh[i], b.il[j], gr[i][j]);
    gi[i][j] = mf(nqh[i], b.rl[j], gi[i][j]);
  }
#pragma unroll
  for (int i = 0; i < MB / 2; ++i) {
    gr[i][j] = mf(a.ql[i], b.ih[j], gr[i][j]);
    gi[i][j] = mf(nql[i], b.rh[j], gi[i][j]);
  }
}

// Scheduling groups for one pipeline step: the next chunk's LDS reads, one per matrix-core
// instruction, then the global->LDS loads spread over the following ones, then the rest.
// The F16F8 path has fewer, longer matrix-core instructions per step than LDS reads and loads
// together: two reads per instruction, then one load per instruction (LOADS_FIRST: the loads
// go first, which gives them the most time to land before the step that waits for them).
// N times: one matrix-core instruction, two LDS reads, one global->LDS load
template <int N>
__device__ __forceinline__ void sched_read_load() {
  if constexpr (N > 0) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
    __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
    sched_read_load<N - 1>();
  }
}

template <int PREC, int MB, int NB, int NVM, int S, bool LOADS_FIRST = false, bool RE = false>
__device__ __forceinline__ void interleave() {
  constexpr int kMFMA = 0x008, kVMEM = 0x010, kDSREAD = 0x100;
  constexpr bool split = PREC == LRS_BF16X2 || PREC == LRS_FP16X2;
  constexpr bool f8 = PREC == LRS_F16F8;
  // instructions per step: LDS reads of 16 bytes, matrix-core instructions (real orbitals:
  // no second fp8 column fragment, and only the products that feed Re G)
  constexpr bool m3 = PREC == LRS_FP64_3M;
  constexpr int NDS = f8 ? (RE ? 2 * MB + 2 * NB : 2 * MB + 3 * NB)
                         : (split ? 2 * (MB + NB) : (m3 ? 6 * (MB + NB) : 4 * (MB + NB)));
  constexpr int NMF0 = f8 ? 3 * MB * NB / 2
                          : (split ? 3 * MB * NB
                                   : (PREC == LRS_FP64 ? 16 * MB * NB : (m3 ? 12 * MB * NB : 32 * MB * NB)));
  constexpr int NMF = RE ? NMF0 / 2 : NMF0;
  constexpr int R = (NMF - NDS) / NVM > 0 ? (NMF - NDS) / NVM : 1;
  if constexpr (f8 && RE) {
    // too few matrix-core instructions for the read pairs and the loads one after the other:
    // a load with each read pair, then the rest
    static_assert(NDS % 2 == 0 && NVM <= NDS / 2 && NDS / 2 <= NMF, "F16F8 real step groups");
    sched_read_load<NVM>();
    sched_pairs<NDS / 2 - NVM, kMFMA, 1, kDSREAD, 2>();
  } else if constexpr (f8 && LOADS_FIRST) {
    static_assert(NDS % 2 == 0 && NDS / 2 + NVM <= NMF, "F16F8 step groups");
    sched_pairs<NVM, kMFMA, 1, kVMEM, 1>();
    sched_pairs<NDS / 2, kMFMA, 1, kDSREAD, 2>();
  } else if constexpr (f8) {
    static_assert(NDS % 2 == 0 && NDS / 2 + NVM <= NMF, "F16F8 step groups");
    sched_pairs<NDS / 2, kMFMA, 1, kDSREAD, 2>();
    sched_pairs<NVM, kMFMA, 1, kVMEM, 1>();
  } else {
    sched_pairs<NDS, kMFMA, 1, kDSREAD, 1>();
    sched_pairs<NVM, kMFMA, R, kVMEM, 1>();
  }
  __builtin_amdgcn_sched_group_barrier(kMFMA, NMF, 0);
}

// Scheduling groups of a rotating step: the next chunk's A reads one per matrix-core
// instruction, the global->LDS loads spread over the rest of block column 0, then per block
// column its matrix-core instructions followed by the refill of its B fragments.
template <int NJ, int NMFJ>
__device__ __forceinline__ void sched_cols() {
  if constexpr (NJ > 0) {
    __builtin_amdgcn_sched_group_barrier(0x008, NMFJ, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
    sched_cols<NJ - 1, NMFJ>();
  }
}
template <int MB, int NB, int NVM>
__device__ __forceinline__ void interleave_rot() {
  constexpr int kMFMA = 0x008, kVMEM = 0x010, kDSREAD = 0x100;
  constexpr int NAR = 2 * MB;          // A reads (16 bytes each)
  constexpr int NMFJ = 6 * MB;         // matrix-core instructions per B block column
  constexpr int R = (NMFJ - NAR) / NVM > 0 ? (NMFJ - NAR) / NVM : 1;
  constexpr int REST = NMFJ - NAR - R * NVM > 0 ? NMFJ - NAR - R * NVM : 0;
  sched_pairs<NAR, kMFMA, 1, kDSREAD, 1>();
  sched_pairs<NVM, kMFMA, R, kVMEM, 1>();
  if constexpr (REST > 0) __builtin_amdgcn_sched_group_barrier(kMFMA, REST, 0);
  __builtin_amdgcn_sched_group_barrier(kDSREAD, 4, 0);
  sched_cols<NB / 2 - 1, NMFJ>();
}

// ----------------------------------------------------------------------------- kernel
// The chunks of a tile (term-major, then K) stream through a ring of S LDS slots, each a
// separate __shared__ array so that the compiler can tell the slots' direct-to-LDS loads
// apart and wait only for the slot it reads.  Chunk q lives in slot q % S.  Per chunk q,
// with chunk q's fragments already in registers:
//   wait for chunk q+1's global->LDS loads and barrier (which also retires chunk q's LDS
//   reads, so slot q % S is free)
//   read chunk q+1's fragments into the other register set
//   start chunk q+S's loads into slot q % S
//   run chunk q's matrix-core instructions
// so the LDS reads of the next chunk and the global loads of the following S-1 chunks overlap
// the matrix-core work.  The chunks of one term run in two phases (occupied then unoccupied
// K), each a multiple of S chunks, so slots and register sets follow a fixed pattern.
template <int PREC, int WMW, int WNW, int MB, int NB, int S, int IL, int ROT, int MODE>
__global__ __launch_bounds__(WMW * WNW * 64) void chi0_kernel(Chi0Params P) {
  using acc_t = typename Prec<PREC>::acc_t;
  static_assert(!ROT || PREC == LRS_BF16X2 || PREC == LRS_FP16X2, "rotating B: split paths");
  // with ROT the register sets hold A fragments only; the B fragments live in `bfr`
  using frag_t = typename std::conditional<ROT != 0, FragsA<PREC, MB>, Frags<PREC, MB, NB>>::type;
  constexpr int TB = Prec<PREC>::TB;
  constexpr int BLK = Prec<PREC>::BLK, ELEMS = Prec<PREC>::ELEMS;
  constexpr int AM = MB * 16 / BLK, AN = NB * 16 / BLK;   // accumulator blocks per wave
  static_assert(AM * BLK == MB * 16 && AN * BLK == NB * 16, "wave tile vs block size");
  constexpr int BM = WMW * MB * 16;
  constexpr int BN = WNW * NB * 16;
  constexpr int A_BYTES = (BM / 16) * TB;
  constexpr int B_BYTES = (BN / 16) * TB;
  constexpr int STAGE = A_BYTES + B_BYTES;
  constexpr int NWAVES = WMW * WNW;
  constexpr int NLOAD = STAGE / 1024;   // 1 KiB wave-wide loads per stage
  constexpr int LPW = NLOAD / NWAVES;   // loads per wave per chunk
  static_assert(NLOAD % NWAVES == 0, "stage split");
  static_assert(S == 2 || S == 4, "ring depth");
  static_assert((S - 2) * LPW <= 63, "vector-memory counter range");
  __shared__ __attribute__((aligned(1024))) unsigned char lds0[STAGE];
  __shared__ __attribute__((aligned(1024))) unsigned char lds1[STAGE];
  __shared__ __attribute__((aligned(1024))) unsigned char lds2[S > 2 ? STAGE : 1024];
  __shared__ __attribute__((aligned(1024))) unsigned char lds3[S > 2 ? STAGE : 1024];
  auto slot = [&](auto I) -> unsigned char* {
    constexpr int i = decltype(I)::value;
    if constexpr (i == 0) return lds0;
    else if constexpr (i == 1) return lds1;
    else if constexpr (i == 2) return lds2;
    else return lds3;
  };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WNW, wn = wave % WNW;
  const int G = gridDim.x;
  const int bslot = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  const int nch = P.nch;
  const int nseq = P.T * nch;

  // global -> LDS: the next chunk to load has its A tiles at `an` and its B tiles at `bn`; the
  // stage's A tiles and B tiles are each one contiguous run, and the wave's share of its 1 KiB
  // pieces goes straight into LDS (lane l's 16 bytes at +16 l).  The A operand is stored
  // [term][chunk][row block], so its chunks follow each other across terms; the B operand has
  // one term's worth of chunks and starts over at each term.
  constexpr int NA = A_BYTES / 1024;
  static_assert(NA % NWAVES == 0, "A pieces per wave");
  const size_t a_step = (size_t)P.a_nrb * TB, b_step = (size_t)P.b_ncb * TB;
  const unsigned char* an = nullptr;
  const unsigned char* bn = nullptr;
  const unsigned char* b0 = nullptr;
  int cn = 0;
  // `more` false (no chunk left in the tile): load the last chunk again, so that every step
  // issues the same loads from in-bounds addresses; the slot it lands in is not read again in
  // this tile, and the next tile's loads into it are issued later, so they land later.
  auto issue_next = [&](unsigned char* dst, bool more) {
    const unsigned char* a = more ? an : an - a_step;
    const unsigned char* b = more ? bn : (cn == 0 ? b0 + (size_t)(nch - 1) * b_step : bn - b_step);
#pragma unroll
    for (int k = 0; k < LPW; ++k) {
      const int j = k * NWAVES + wave;
      const unsigned char* src = k * NWAVES < NA ? a + j * 1024 : b + (j - NA) * 1024;
      __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1)))*)src,
                                       (void __attribute__((address_space(3)))*)(dst + j * 1024),
                                       16, 0, 0);
    }
    // advance without a branch, so that the step stays one basic block
    const int c1 = cn + 1;
    const bool wrap = more && c1 == nch;
    an = more ? an + a_step : an;
    bn = wrap ? b0 : (more ? bn + b_step : bn);
    cn = wrap ? 0 : (more ? c1 : cn);
  };
  // in steady state the loads of chunks q+2 .. q+S-1 may still be in flight at step q
  constexpr int kKeep = (S - 2) * LPW;

  // G_o of the current term waits here (one slot per workgroup) while G_u accumulates.
  // Addresses used once per term are rebuilt from opaque copies of their inputs inside the term
  // loop, so that the compiler does not hoist them and keep them live across the chunk loop.
  auto opaque = [](int x) {
    asm volatile("" : "+v"(x));
    return x;
  };
  auto park_at = [&](int ln, int i, int j, int comp) -> acc_t* {
    acc_t* park = (acc_t*)(P.park + (size_t)blockIdx.x * NWAVES * AM * AN * 2 * 64 * sizeof(acc_t));
    return park + (((size_t)(wave * AM + i) * AN + j) * 2 + comp) * 64 + ln;
  };

  // The workgroups of one XCD (b % 8) share their tiles' operand panels in that XCD's L2 only
  // while they run the same stretch of K.  Left alone they drift apart over the launch, and
  // the panels are fetched again; with P.sync they meet at every term start: each adds one to
  // its group's counter and waits (a bounded spin, so a group member that never arrives
  // delays but cannot stall the launch) until every member with a tile in this round has
  // arrived.  Member count of a round: the group's tiles that exist.
  const int grp = blockIdx.x & 7, gsz = G >> 3;
  unsigned int done = 0;          // this group's term starts before the current tile
  for (long long tau = bslot; tau < P.ntiles; tau += G) {
    const TileDesc td = P.tiles[tau];
    const long long base = tau - (blockIdx.x >> 3);   // the group's first tile this round
    const unsigned int members = (unsigned int)max(0LL, min((long long)gsz, P.ntiles - base));
    acc_t gr[AM][AN], gi[AM][AN];
    // the third product of the 3M form (FP64 3M only; a placeholder otherwise)
    acc_t gx[PREC == LRS_FP64_3M ? AM : 1][PREC == LRS_FP64_3M ? AN : 1];
    frag_t fa, fb;
    FragsB<PREC, NB> bfr;

    ring_barrier<63>();              // the previous tile is done reading every slot
    an = P.a + (size_t)(td.a_row0 >> 4) * TB + lane * 16;
    b0 = P.b + (size_t)(td.b_col0 >> 4) * TB + lane * 16;
    bn = b0;
    cn = 0;
    // every phase holds a multiple of S chunks, so the tile has at least S
    issue_next(slot(std::integral_constant<int, 0>{}), true);
    issue_next(slot(std::integral_constant<int, 1>{}), true);
    if constexpr (S > 2) {
      issue_next(slot(std::integral_constant<int, 2>{}), true);
      issue_next(slot(std::integral_constant<int, 3>{}), true);
    }
    ring_barrier<0>();
    {
      const unsigned char* s0 = slot(std::integral_constant<int, 0>{});
      if constexpr (ROT) {
        load_a_split<PREC, MB>(s0 + wm * MB * TB, lane, fa);
#pragma unroll
        for (int j = 0; j < NB / 2; ++j)
          load_b_split<PREC, NB>(s0 + A_BYTES + wn * NB * TB, lane, j, bfr);
      } else {
        load_frags<PREC, MB, NB, MODE == 3>(s0 + wm * MB * TB, s0 + A_BYTES + wn * NB * TB, lane, fa);
      }
    }
    int q = 0;
    // chunk q (in slot I = q % S) with its fragments in `cur`; the next chunk's fragments go
    // to `nxt`.  Every step issues LPW loads per wave, so at step q the loads of chunks
    // q+2 .. q+S-1 are the last kKeep; `full` asks for a complete drain instead (first chunk of
    // a phase, after the previous phase's global stores).
    auto step = [&](auto I, frag_t& cur, frag_t& nxt, bool full) {
      constexpr int i = decltype(I)::value;
      constexpr int inext = (i + 1) % S;
      if (full) ring_barrier<0>();
      else ring_barrier<kKeep>();
      // (after the tile's last chunk these fragments are read but not used)
      const unsigned char* sn = slot(std::integral_constant<int, inext>{});
      if constexpr (ROT) {
        load_a_split<PREC, MB>(sn + wm * MB * TB, lane, nxt);
        issue_next(slot(I), q + S < nseq);
#pragma unroll
        for (int j = 0; j < NB / 2; ++j) {
          mma_col_split<PREC, MB, NB>(cur, bfr, j, gr, gi);
          load_b_split<PREC, NB>(sn + A_BYTES + wn * NB * TB, lane, j, bfr);
        }
        interleave_rot<MB, NB, LPW>();
      } else {
        load_frags<PREC, MB, NB, MODE == 3>(sn + wm * MB * TB, sn + A_BYTES + wn * NB * TB, lane, nxt);
        issue_next(slot(I), q + S < nseq);
        if constexpr (IL == 0) {
          // LDS reads and loads first, then the matrix-core block
          __builtin_amdgcn_sched_barrier(0);
          if constexpr (PREC == LRS_FP64_3M) mma_frags_3m<MB, NB>(cur, gr, gi, gx);
          else if constexpr (MODE == 3) mma_frags_re<PREC, MB, NB>(cur, gr);
          else mma_frags<PREC, MB, NB>(cur, gr, gi);
        } else {
          // LDS reads and loads spread between the matrix-core instructions
          if constexpr (PREC == LRS_FP64_3M) mma_frags_3m<MB, NB>(cur, gr, gi, gx);
          else if constexpr (MODE == 3) mma_frags_re<PREC, MB, NB>(cur, gr);
          else mma_frags<PREC, MB, NB>(cur, gr, gi);
          interleave<PREC, MB, NB, LPW, S, IL == 2, MODE == 3>();
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      ++q;
    };
    // one ring cycle: S chunks starting at slot 0
    auto cycle = [&](bool first) {
      step(std::integral_constant<int, 0>{}, fa, fb, first);
      step(std::integral_constant<int, 1>{}, fb, fa, false);
      if constexpr (S > 2) {
        step(std::integral_constant<int, 2 % S>{}, fa, fb, false);
        step(std::integral_constant<int, 3 % S>{}, fb, fa, false);
      }
    };
    auto zero = [&] {
#pragma unroll
      for (int i = 0; i < AM; ++i)
#pragma unroll
        for (int j = 0; j < AN; ++j) {
          gr[i][j] = zero_acc<acc_t>();
          gi[i][j] = zero_acc<acc_t>();
          if constexpr (PREC == LRS_FP64_3M) gx[i][j] = zero_acc<acc_t>();
        }
    };
    for (int t = 0; t < P.T; ++t) {
      if (P.sync) {
        if (tid == 0) {
          unsigned int* ctr = P.sync + grp * 16;
          const unsigned int target = done + (unsigned int)(t + 1) * members;
          __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          for (int it = 0; it < 512; ++it) {   // at most about half a millisecond
            if (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            __builtin_amdgcn_s_sleep(4);
          }
        }
        __builtin_amdgcn_s_barrier();
      }
      zero();
      for (int ch = 0; ch < P.nch_o; ch += S) cycle(ch == 0);
      if constexpr (PREC == LRS_FP64_3M) combine_3m<MB, NB>(gr, gi, gx);
      {
        const int ln = opaque(lane);
#pragma unroll
        for (int i = 0; i < AM; ++i)
#pragma unroll
          for (int j = 0; j < AN; ++j) {
            *park_at(ln, i, j, 0) = gr[i][j];
            *park_at(ln, i, j, 1) = gi[i][j];
          }
      }
      zero();
      for (int ch = P.nch_o; ch < nch; ch += S) cycle(ch == P.nch_o);
      if constexpr (PREC == LRS_FP64_3M) combine_3m<MB, NB>(gr, gi, gx);
      // here gr, gi hold G_u; G_o comes back block by block.  Per accumulator block every
      // global load is issued before the first use (elements outside the output take the
      // tile origin's address and skip the store), so the block costs one memory latency.
      const int ln = opaque(lane);
      const long long obase = td.out_off + opaque(0);
#pragma unroll
      for (int i = 0; i < AM; ++i)
#pragma unroll
        for (int j = 0; j < AN; ++j) {
          const acc_t or_ = *park_at(ln, i, j, 0), oi_ = *park_at(ln, i, j, 1);
          int off[ELEMS], dg[ELEMS];
          bool in[ELEMS];
#pragma unroll
          for (int e = 0; e < ELEMS; ++e) {
            int rr, cc;
            elem_rc<PREC>(ln, e, rr, cc);
            const int row = wm * MB * 16 + i * BLK + rr;
            const int col = wn * NB * 16 + j * BLK + cc;
            in[e] = row < td.nrows && col < td.ncols;
            off[e] = in[e] ? row * td.ldo + col : 0;
            dg[e] = col - row - td.pad;   // (site column) - (site row), adjoint mode
          }
          if constexpr (MODE == 1 || MODE == 2) {
            // adjoint: Hu = lam * conj(G_u), Ho = lam * conj(G_o) on a site block.  lam is
            // symmetric (or the coefficient matrix Hermitian) and G Hermitian there, so
            // H(c, r) = conj(H(r, c)): the host lists only tiles that reach the upper
            // triangle, each element on or above the diagonal is stored with its conjugate at
            // the transposed place, and each place is written once.
            double l[ELEMS], la[ELEMS];
#pragma unroll
            for (int e = 0; e < ELEMS; ++e) l[e] = P.lam[obase + off[e]];
            if (P.lam_a) {
#pragma unroll
              for (int e = 0; e < ELEMS; ++e) la[e] = P.lam_a[obase + off[e]];
            }
#pragma unroll
            for (int e = 0; e < ELEMS; ++e)
              if (in[e] && dg[e] >= 0) {
                const long long o = obase + off[e];
                double hur = l[e] * (double)gr[i][j][e], hui = -l[e] * (double)gi[i][j][e];
                double hor = l[e] * (double)or_[e], hoi = -l[e] * (double)oi_[e];
                if (P.lam_a) {
                  // (a + i b) conj(g) with a = adj_c lam, b = +-adj_s lam_a
                  const double a = P.adj_c * l[e], b = P.adj_s * la[e];
                  const double ur = gr[i][j][e], ui = gi[i][j][e];
                  const double vr = or_[e], vi = oi_[e];
                  hur = a * ur + b * ui;
                  hui = b * ur - a * ui;
                  hor = a * vr - b * vi;
                  hoi = -b * vr - a * vi;
                }
                if constexpr (MODE == 1) {
                  const long long ot = o + (long long)dg[e] * (td.ldo - 1);
                  P.hu_re[o] = hur;
                  P.hu_im[o] = hui;
                  P.ho_re[o] = hor;
                  P.ho_im[o] = hoi;
                  if (dg[e] > 0) {
                    P.hu_re[ot] = hur;
                    P.hu_im[ot] = -hui;
                    P.ho_re[ot] = hor;
                    P.ho_im[ot] = -hoi;
                  }
                } else {
                  // (p, r) in the block: row and column offsets of the tile plus the element's
                  int rr, cc;
                  elem_rc<PREC>(ln, e, rr, cc);
                  const int pr = td.m0 + wm * MB * 16 + i * BLK + rr;
                  const int pc = td.c0 + wn * NB * 16 + j * BLK + cc;
                  // (block base: out_off counts one value per element, the tiles four)
                  const long long hb = 4 * (td.out_off - ((long long)td.m0 * td.ldo + td.c0));
                  const long long ht = hb + h_tile_offset(pr, pc, td.ldo);
                  put_split(P.hs_u, 512, ht, hur, hui);
                  put_split(P.hs_o, 512, ht, hor, hoi);
                  if (dg[e] > 0) {
                    const long long htt = hb + h_tile_offset(pc, pr, td.ldo);
                    put_split(P.hs_u, 512, htt, hur, -hui);
                    put_split(P.hs_o, 512, htt, hor, -hoi);
                  }
                }
              }
          } else {
            // chi accumulates across terms in FP64 in the output itself (this tile's entries
            // belong to this workgroup only); the last term applies the prefactor.  On a site
            // block chi0 is symmetric (G Hermitian, so Re[G_o conj(G_u)] is the same at (r, c)
            // and (c, r)): the host lists only tiles that reach the upper triangle, and each
            // element on or above the diagonal is stored at both places
            const double ct = P.c[t];
            const double cti = P.ci ? P.ci[t] : 0.0;
            const double scale = t == P.T - 1 ? P.pref : 1.0;
            double old[ELEMS];
            if (t > 0) {
#pragma unroll
              for (int e = 0; e < ELEMS; ++e) old[e] = P.out[obase + off[e]];
            } else {
#pragma unroll
              for (int e = 0; e < ELEMS; ++e) old[e] = 0.0;
            }
#pragma unroll
            for (int e = 0; e < ELEMS; ++e) {
              // Re[(c + i c_i) G_o conj(G_u)]; c_i is zero but for imaginary frequency
              const double v = ct * ((double)or_[e] * (double)gr[i][j][e] +
                                     (double)oi_[e] * (double)gi[i][j][e]) -
                               cti * ((double)oi_[e] * (double)gr[i][j][e] -
                                      (double)or_[e] * (double)gi[i][j][e]);
              const double r = (v + old[e]) * scale;
              if (in[e] && (!P.sym || dg[e] >= 0)) {
                P.out[obase + off[e]] = r;
                if (P.sym && dg[e] > 0) P.out[obase + off[e] + (long long)dg[e] * (td.ldo - 1)] = r;
              }
            }
            if (P.keep_o) {
              const long long kb = (long long)t * P.keep_stride + obase;
#pragma unroll
              for (int e = 0; e < ELEMS; ++e)
                if (in[e] && dg[e] >= 0) {
                  if constexpr (PREC == LRS_FP64 || PREC == LRS_FP64_3M) {
                    ((double2*)P.keep_o)[kb + off[e]] = double2{(double)or_[e], (double)oi_[e]};
                    ((double2*)P.keep_u)[kb + off[e]] =
                        double2{(double)gr[i][j][e], (double)gi[i][j][e]};
                  } else {
                    ((float2*)P.keep_o)[kb + off[e]] = float2{(float)or_[e], (float)oi_[e]};
                    ((float2*)P.keep_u)[kb + off[e]] =
                        float2{(float)gr[i][j][e], (float)gi[i][j][e]};
                  }
                }
            }
          }
        }
    }
    done += (unsigned int)P.T * members;
  }
}

// variant table: {WMW, WNW, MB, NB, S, IL, ROT}; S = LDS ring slots, IL = 1 interleaves the LDS
// reads and loads with the matrix-core instructions, ROT = 1 rotates the B fragments (split
// paths; allows the 128 x 64 wave tile).  Split paths: 128 x 128 workgroup tiles with four
// slots (default), 128 x 256 with two slots, 128 x 256 from 128 x 64 wave tiles, and
// 128 x 192 (four 40 KiB slots fill the 160 KiB of LDS).
template <int PREC, int V>
struct Variant;
#define LRS_VARIANT(PR, V, A, B, C, D, E, F, G)                         \
  template <>                                                          \
  struct Variant<PR, V> {                                              \
    static constexpr int WMW = A, WNW = B, MB = C, NB = D, S = E, IL = F, ROT = G; \
  };
LRS_VARIANT(LRS_FP64, 0, 2, 2, 2, 4, 2, 1, 0)
LRS_VARIANT(LRS_FP64, 1, 2, 2, 2, 2, 4, 1, 0)
LRS_VARIANT(LRS_FP64, 2, 2, 2, 2, 2, 4, 0, 0)
LRS_VARIANT(LRS_FP64, 3, 2, 2, 2, 4, 2, 0, 0)
LRS_VARIANT(LRS_FP32, 0, 2, 2, 2, 2, 4, 1, 0)
LRS_VARIANT(LRS_FP32, 1, 2, 2, 2, 4, 2, 1, 0)
LRS_VARIANT(LRS_FP32, 2, 2, 2, 2, 4, 2, 0, 0)
LRS_VARIANT(LRS_FP32, 3, 2, 2, 2, 2, 4, 0, 0)
LRS_VARIANT(LRS_BF16X2, 0, 2, 2, 4, 4, 4, 1, 0)
LRS_VARIANT(LRS_BF16X2, 1, 2, 2, 4, 8, 2, 1, 0)
LRS_VARIANT(LRS_BF16X2, 2, 1, 4, 8, 4, 2, 1, 1)
LRS_VARIANT(LRS_BF16X2, 3, 2, 2, 4, 6, 4, 1, 0)
LRS_VARIANT(LRS_FP16X2, 0, 2, 2, 4, 4, 4, 1, 0)
LRS_VARIANT(LRS_FP16X2, 1, 2, 2, 4, 8, 2, 1, 0)
LRS_VARIANT(LRS_FP16X2, 2, 1, 4, 8, 4, 2, 1, 1)
LRS_VARIANT(LRS_FP16X2, 3, 2, 2, 4, 6, 4, 1, 0)
// F16F8: 40 KiB (128 x 192) or 32 KiB (128 x 128) stages of 16 K, four-slot ring, interleaved
// or not.  The wider tile moves a third fewer operand bytes per matrix-core cycle and is the
// faster one on the precision workload (2.55 s against 2.94 s for its site x grid launch).
LRS_VARIANT(LRS_F16F8, 0, 2, 2, 4, 6, 4, 1, 0)
LRS_VARIANT(LRS_F16F8, 1, 2, 2, 4, 4, 4, 1, 0)
LRS_VARIANT(LRS_F16F8, 2, 2, 2, 4, 6, 4, 2, 0)
LRS_VARIANT(LRS_F16F8, 3, 2, 2, 4, 4, 4, 0, 0)
// FP64 3M: a third accumulator and operand plane per block, so 32 x 32 or 32 x 48 wave tiles
// (stages of 48 KiB for 64 x 64, 60 KiB for 64 x 96: two slots)
LRS_VARIANT(LRS_FP64_3M, 0, 2, 2, 2, 3, 2, 1, 0)
LRS_VARIANT(LRS_FP64_3M, 1, 2, 2, 2, 2, 2, 1, 0)
LRS_VARIANT(LRS_FP64_3M, 2, 2, 2, 2, 3, 2, 0, 0)
LRS_VARIANT(LRS_FP64_3M, 3, 2, 2, 2, 2, 2, 0, 0)
#undef LRS_VARIANT
constexpr int kNumVariants = 4;

template <int PREC, int V>
constexpr int lds_bytes_v() {
  using Vt = Variant<PREC, V>;
  return Vt::S * (Vt::WMW * Vt::MB + Vt::WNW * Vt::NB) * Prec<PREC>::TB;
}

template <int PREC, int V>
constexpr size_t park_bytes_v() {
  using Vt = Variant<PREC, V>;
  return (size_t)Vt::WMW * Vt::WNW * (Vt::MB * 16 / Prec<PREC>::BLK) *
         (Vt::NB * 16 / Prec<PREC>::BLK) * 2 * 64 * sizeof(typename Prec<PREC>::acc_t);
}

template <int PREC, int V, int MODE>
constexpr auto kernel_v() {
  using Vt = Variant<PREC, V>;
  static_assert(lds_bytes_v<PREC, V>() <= 160 * 1024, "LDS ring too large");
  return &chi0_kernel<PREC, Vt::WMW, Vt::WNW, Vt::MB, Vt::NB, Vt::S, Vt::IL, Vt::ROT, MODE>;
}

template <int PREC, int V, int MODE>
hipError_t launch_v(int grid, const Chi0Params& P, hipStream_t s) {
  using Vt = Variant<PREC, V>;
  constexpr auto k = kernel_v<PREC, V, MODE>();
  hipLaunchKernelGGL(k, dim3(grid), dim3(Vt::WMW * Vt::WNW * 64), 0, s, P);
  return hipGetLastError();
}

template <int PREC, int MODE = 0>
hipError_t launch_p(int variant, int grid, const Chi0Params& P, hipStream_t s) {
  switch (variant) {
    case 0: return launch_v<PREC, 0, MODE>(grid, P, s);
    case 1: return launch_v<PREC, 1, MODE>(grid, P, s);
    case 2: return launch_v<PREC, 2, MODE>(grid, P, s);
    case 3: return launch_v<PREC, 3, MODE>(grid, P, s);
  }
  return hipErrorInvalidValue;
}

template <int PREC, int V>
TileShape shape_v() {
  using Vt = Variant<PREC, V>;
  return TileShape{Vt::WMW * Vt::MB * 16, Vt::WNW * Vt::NB * 16, Vt::WMW * Vt::WNW * 64,
                   park_bytes_v<PREC, V>()};
}
template <int PREC>
TileShape shape_p(int v) {
  switch (v) {
    case 0: return shape_v<PREC, 0>();
    case 1: return shape_v<PREC, 1>();
    case 2: return shape_v<PREC, 2>();
    default: return shape_v<PREC, 3>();
  }
}

template <int PREC>
bool rot_p(int v) {
  switch (v) {
    case 0: return Variant<PREC, 0>::ROT != 0;
    case 1: return Variant<PREC, 1>::ROT != 0;
    case 2: return Variant<PREC, 2>::ROT != 0;
    default: return Variant<PREC, 3>::ROT != 0;
  }
}

template <int PREC, int V>
int occ_v() {
  using Vt = Variant<PREC, V>;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, reinterpret_cast<const void*>(kernel_v<PREC, V, 0>()), Vt::WMW * Vt::WNW * 64, 0) !=
      hipSuccess)
    return 1;
  return n;
}
template <int PREC>
int occ_p(int v) {
  switch (v) {
    case 0: return occ_v<PREC, 0>();
    case 1: return occ_v<PREC, 1>();
    case 2: return occ_v<PREC, 2>();
    default: return occ_v<PREC, 3>();
  }
}

template <int PREC>
hipError_t prep_p(const double* site, int rows_pad, int K_pad, const int* slot_row, int rb0,
                  int nrb, const double* w, int w_stride, int q_woff, int t0, int nt,
                  double a_scale, void* out, hipStream_t s) {
  if constexpr (PREC == LRS_F16F8) {
    const long long n = (long long)nrb * (K_pad / 16) * 32;
    hipLaunchKernelGGL(prep_site_f16f8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       s, site, rows_pad, K_pad, slot_row, rb0, nrb, w, w_stride, q_woff, t0,
                       nt, a_scale, (unsigned char*)out);
    return hipGetLastError();
  }
  const int nch = K_pad / Prec<PREC>::KC;
  const int slots = (PREC == LRS_BF16X2 || PREC == LRS_FP16X2) ? 32 : 64;
  const long long n = (long long)nrb * nch * slots;
  hipLaunchKernelGGL(prep_site_kernel<PREC>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     site, rows_pad, K_pad, slot_row, rb0, nrb, w, w_stride, q_woff, t0, nt,
                     a_scale, (unsigned char*)out);
  return hipGetLastError();
}

}  // namespace

int chi0_num_variants(int prec) { return kNumVariants; }

// fastest variant measured on the precision workload (the tuner can override it)
int chi0_default_variant(int) { return 0; }

int chi0_blocks_per_cu(int prec, int variant) {
  switch (prec) {
    case LRS_FP64: return occ_p<LRS_FP64>(variant);
    case LRS_FP32: return occ_p<LRS_FP32>(variant);
    case LRS_BF16X2: return occ_p<LRS_BF16X2>(variant);
    case LRS_F16F8: return occ_p<LRS_F16F8>(variant);
    case LRS_FP64_3M: return occ_p<LRS_FP64_3M>(variant);
    default: return occ_p<LRS_FP16X2>(variant);
  }
}

bool chi0_variant_rotates(int prec, int variant) {
  switch (prec) {
    case LRS_BF16X2: return rot_p<LRS_BF16X2>(variant);
    case LRS_FP16X2: return rot_p<LRS_FP16X2>(variant);
    default: return false;
  }
}

TileShape chi0_shape(int prec, int variant) {
  switch (prec) {
    case LRS_FP64: return shape_p<LRS_FP64>(variant);
    case LRS_FP32: return shape_p<LRS_FP32>(variant);
    case LRS_BF16X2: return shape_p<LRS_BF16X2>(variant);
    case LRS_F16F8: return shape_p<LRS_F16F8>(variant);
    case LRS_FP64_3M: return shape_p<LRS_FP64_3M>(variant);
    default: return shape_p<LRS_FP16X2>(variant);
  }
}

hipError_t launch_prep_site(int prec, const double* site, int rows_pad, int K_pad,
                            const int* slot_row, int rb0, int nrb, const double* w,
                            int w_stride, int q_woff, int t0, int nt, double a_scale, void* out,
                            hipStream_t s) {
#define LRS_PREP(PR) \
  prep_p<PR>(site, rows_pad, K_pad, slot_row, rb0, nrb, w, w_stride, q_woff, t0, nt, a_scale, out, s)
  switch (prec) {
    case LRS_FP64: return LRS_PREP(LRS_FP64);
    case LRS_FP32: return LRS_PREP(LRS_FP32);
    case LRS_BF16X2: return LRS_PREP(LRS_BF16X2);
    case LRS_FP16X2: return LRS_PREP(LRS_FP16X2);
    case LRS_F16F8: return LRS_PREP(LRS_F16F8);
    case LRS_FP64_3M: return LRS_PREP(LRS_FP64_3M);
  }
#undef LRS_PREP
  return hipErrorInvalidValue;
}

hipError_t launch_chi0(int prec, int variant, int grid, const void* a_tiles, int a_nrb,
                       const void* b_tiles, int b_ncb, int nch, const double* c,
                       const double* ci, int T, int nch_o, const TileDesc* tiles, int ntiles,
                       double* out, double pref, int sym, unsigned int* sync, void* park,
                       int real, void* keep_o, void* keep_u, long long keep_stride,
                       hipStream_t s) {
  Chi0Params P;
  P.keep_o = keep_o;
  P.keep_u = keep_u;
  P.keep_stride = keep_stride;
  P.ci = ci;
  P.sym = sym;
  P.sync = sync;
  P.park = (unsigned char*)park;
  P.a = (const unsigned char*)a_tiles;
  P.a_nrb = a_nrb;
  P.b = (const unsigned char*)b_tiles;
  P.b_ncb = b_ncb;
  P.nch = nch;
  P.c = c;
  P.T = T;
  P.nch_o = nch_o;
  P.tiles = tiles;
  P.ntiles = ntiles;
  P.out = out;
  P.pref = pref;
  P.lam = nullptr;
  P.lam_a = nullptr;
  P.adj_c = P.adj_s = 0.0;
  P.hu_re = P.hu_im = P.ho_re = P.ho_im = nullptr;
  P.hs_u = P.hs_o = nullptr;
  if (real) {
    switch (prec) {
      case LRS_FP64: return launch_p<LRS_FP64, 3>(variant, grid, P, s);
      case LRS_F16F8: return launch_p<LRS_F16F8, 3>(variant, grid, P, s);
    }
    return hipErrorInvalidValue;
  }
  switch (prec) {
    case LRS_FP64: return launch_p<LRS_FP64>(variant, grid, P, s);
    case LRS_FP32: return launch_p<LRS_FP32>(variant, grid, P, s);
    case LRS_BF16X2: return launch_p<LRS_BF16X2>(variant, grid, P, s);
    case LRS_FP16X2: return launch_p<LRS_FP16X2>(variant, grid, P, s);
    case LRS_F16F8: return launch_p<LRS_F16F8>(variant, grid, P, s);
    case LRS_FP64_3M: return launch_p<LRS_FP64_3M>(variant, grid, P, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_green_adjoint(int prec, int grid, const void* a_tiles, int a_nrb,
                                const void* b_tiles, int b_ncb, int nch, const double* c,
                                int nch_o, const TileDesc* tiles, int ntiles, const double* lam,
                                const double* lam_a, double adj_c, double adj_s,
                                double* hu_re, double* hu_im, double* ho_re, double* ho_im,
                                void* hs_u, void* hs_o, void* park, hipStream_t s) {
  Chi0Params P;
  P.keep_o = P.keep_u = nullptr;
  P.keep_stride = 0;
  P.park = (unsigned char*)park;
  P.a = (const unsigned char*)a_tiles;
  P.a_nrb = a_nrb;
  P.b = (const unsigned char*)b_tiles;
  P.b_ncb = b_ncb;
  P.nch = nch;
  P.c = c;
  P.ci = nullptr;
  P.T = 1;
  P.nch_o = nch_o;
  P.tiles = tiles;
  P.ntiles = ntiles;
  P.out = nullptr;
  P.pref = 1.0;
  P.sym = 0;
  P.sync = nullptr;
  P.lam = lam;
  P.lam_a = lam_a;
  P.adj_c = adj_c;
  P.adj_s = adj_s;
  P.hu_re = hu_re;
  P.hu_im = hu_im;
  P.ho_re = ho_re;
  P.ho_im = ho_im;
  P.hs_u = (__bf16*)hs_u;
  P.hs_o = (__bf16*)hs_o;
  switch (prec) {
    case LRS_FP64: return launch_v<LRS_FP64, 0, 1>(grid, P, s);
    case LRS_BF16X2: return launch_v<LRS_BF16X2, 0, 2>(grid, P, s);
    case LRS_F16F8: return launch_v<LRS_F16F8, 1, 2>(grid, P, s);
  }
  return hipErrorInvalidValue;
}

namespace {
// The adjoint's H = (coefficient matrix) o conj(G) from one term's kept Green's functions, the
// same arithmetic and values as the mode-2 epilogue.  One workgroup per operand-tile piece (32
// block rows p x 16 block columns r, four planes of 512 values), element e of each plane at
// p = 32 (piece row) + (e / 8) % 32, r = 16 (piece column) + 8 (e / 256) + e % 8, so each wave
// writes whole runs of a plane.  G is kept on and above the diagonal only; H is Hermitian, so
// below it H(p, r) = conj(H(r, p)), formed from the transposed element.
__global__ __launch_bounds__(512) void h_from_kept_kernel(
    const float2* keep_o, const float2* keep_u, const long long* blk_off,
    const long long* pblk_off, const int* blk_n, const double* lam, const double* lam_a,
    double adj_c, double adj_s, __bf16* hs_u, __bf16* hs_o) {
  const int st = blockIdx.y;
  const int n = blk_n[st];
  const int np = site_block_ld(n, 1);
  const int npr = np >> 5, npc = np >> 4;            // pieces along p and along r
  const int piece = blockIdx.x;
  if (piece >= npr * npc) return;
  const int pb = piece % npr, rb = piece / npr;
  const int e = threadIdx.x;
  const int p = pb * 32 + ((e >> 3) & 31), r = rb * 16 + ((e >> 8) << 3) + (e & 7);
  if (p >= n || r >= n) return;                     // padding stays zero
  const bool up = r >= p;
  const int a = up ? p : r, b = up ? r : p;         // the kept element (a <= b)
  const long long kk = blk_off[st] + (long long)a * n + b;
  const long long lk = pblk_off[st] + (long long)a * np + b;
  const float2 go = keep_o[kk], gu = keep_u[kk];
  const double l = lam[lk];
  double hur = l * (double)gu.x, hui = -l * (double)gu.y;
  double hor = l * (double)go.x, hoi = -l * (double)go.y;
  if (lam_a) {
    const double ac = adj_c * l, bs = adj_s * lam_a[lk];
    const double ur = gu.x, ui = gu.y, vr = go.x, vi = go.y;
    hur = ac * ur + bs * ui;
    hui = bs * ur - ac * ui;
    hor = ac * vr - bs * vi;
    hoi = -bs * vr - ac * vi;
  }
  if (!up) {
    hui = -hui;
    hoi = -hoi;
  }
  const long long ht = 4 * pblk_off[st] + ((long long)(rb * npr + pb) << 11) + e;
  put_split(hs_u, 512, ht, hur, hui);
  put_split(hs_o, 512, ht, hor, hoi);
}
}  // namespace

hipError_t launch_h_from_kept(const void* keep_o, const void* keep_u, int nsites,
                              const long long* blk_off, const long long* pblk_off,
                              const int* blk_n, const int* blk_n_host, const double* lam,
                              const double* lam_a,
                              double adj_c, double adj_s, void* hs_u, void* hs_o,
                              hipStream_t s) {
  int npmax = 0;
  for (int i = 0; i < nsites; ++i) {
    const int np = site_block_ld(blk_n_host[i], 1);
    npmax = np > npmax ? np : npmax;
  }
  const int pieces = (npmax >> 5) * (npmax >> 4);
  hipLaunchKernelGGL(h_from_kept_kernel, dim3(pieces, nsites), dim3(512), 0, s,
                     (const float2*)keep_o, (const float2*)keep_u, blk_off, pblk_off, blk_n, lam,
                     lam_a, adj_c, adj_s, (__bf16*)hs_u, (__bf16*)hs_o);
  return hipGetLastError();
}

namespace {
// The FP64 adjoint's H planes (hu_re, hu_im, ho_re, ho_im, each site block row-major with the
// padded row stride) from one term's kept FP64 Green's functions, the same values as the
// mode-1 epilogue: one thread per block element, the element on or above the diagonal from
// the kept G, the one below as the conjugate of its transpose (H is Hermitian).
__global__ __launch_bounds__(256) void h_from_kept_f64_kernel(
    const double2* keep_o, const double2* keep_u, const long long* blk_off,
    const long long* pblk_off, const int* blk_n, const double* lam, const double* lam_a,
    double adj_c, double adj_s, double* hu_re, double* hu_im, double* ho_re, double* ho_im) {
  const int st = blockIdx.y;
  const int n = blk_n[st];
  const int np = site_block_ld(n, 1);
  const long long nn = (long long)n * n;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nn;
       q += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(q / n), r = (int)(q - (long long)p * n);
    const bool up = r >= p;
    const int a = up ? p : r, b = up ? r : p;
    const long long kk = blk_off[st] + (long long)a * n + b;
    const long long lk = pblk_off[st] + (long long)a * np + b;
    const double2 go = keep_o[kk], gu = keep_u[kk];
    const double l = lam[lk];
    double hur = l * gu.x, hui = -l * gu.y;
    double hor = l * go.x, hoi = -l * go.y;
    if (lam_a) {
      const double ac = adj_c * l, bs = adj_s * lam_a[lk];
      hur = ac * gu.x + bs * gu.y;
      hui = bs * gu.x - ac * gu.y;
      hor = ac * go.x - bs * go.y;
      hoi = -bs * go.x - ac * go.y;
    }
    if (!up) {
      hui = -hui;
      hoi = -hoi;
    }
    const long long o = pblk_off[st] + (long long)p * np + r;
    hu_re[o] = hur;
    hu_im[o] = hui;
    ho_re[o] = hor;
    ho_im[o] = hoi;
  }
}
}  // namespace

hipError_t launch_h_from_kept_f64(const void* keep_o, const void* keep_u, int nsites,
                                  const long long* blk_off, const long long* pblk_off,
                                  const int* blk_n, const double* lam, const double* lam_a,
                                  double adj_c, double adj_s, double* hu_re, double* hu_im,
                                  double* ho_re, double* ho_im, hipStream_t s) {
  hipLaunchKernelGGL(h_from_kept_f64_kernel, dim3(4096, nsites), dim3(256), 0, s,
                     (const double2*)keep_o, (const double2*)keep_u, blk_off, pblk_off, blk_n,
                     lam, lam_a, adj_c, adj_s, hu_re, hu_im, ho_re, ho_im);
  return hipGetLastError();
}

}  // namespace lrs
