// Adjoint of chi0 on site x site blocks, in FP64 or with split bfloat16 products.
//
// With P_f = -2 s / N_k^2, Lambda = dL/dchi0 (symmetrised: chi0 on a square block is symmetric)
// and per term l the weighted Green's functions G_o^l, G_u^l of the forward pass,
//   dL/dpsi_K (K occupied)   = 2 P_f sum_l c_l alpha_l(K) [ (Lambda o conj(G_u^l)) psi_K ]
//   dL/dpsi_K (K unoccupied) = 2 P_f sum_l c_l beta_l(K)  [ (Lambda o conj(G_o^l)) psi_K ]
//   dL/de_K = P_f sum_l c_l (d weight_l(K)/d e_K) Re[ psi_K^H (Lambda o conj(G^l)) psi_K ]
// (complex gradients as dL/dRe + i dL/dIm; mu and the nodes held fixed).  With complex term
// coefficients c_l + i s_l (chi0 at imaginary frequency, whose site block is not symmetric)
// Lambda splits into its symmetric part Ls and antisymmetric part La, and c_l Lambda becomes
// the Hermitian c_l Ls + i s_l La next to conj(G_u) and c_l Ls - i s_l La next to conj(G_o);
// the energy partials take the real part as before.  Each term's G's are
// recomputed on the matrix cores (the chi0 kernel in an adjoint mode writes
// Lambda o conj(G) directly); the products with psi run as a complex MFMA GEMM (FP64, or
// bfloat16 hi + lo with FP32 accumulation) whose epilogue accumulates the orbital gradient and
// per-row-tile energy partials in FP64.  Every output element has one owner per launch and
// launches are ordered, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "lrs_internal.h"
#include "cgemm64.h"
#include "ring.h"

namespace lrs {
namespace {

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;

struct BwdTile {
  int site_row0;       // first global row of the site
  int r0;              // first local row of this tile
  int ns;              // points of the site
  int k0;              // first K column of this tile
  long long h_off;     // offset of the site's block in the H arrays (FP64: row stride npad; split:
                       // operand tiles, four values per element)
  int part_row;        // row-tile index for the energy partials
  int npad;            // ns rounded up to 64: row stride of the H block, contraction length
  int srow0;           // split GEMM: first slot row of the site in the split psi operand
};

struct BwdParams {
  const double* hu_re;
  const double* hu_im;
  const double* ho_re;
  const double* ho_im;
  const double* psi;     // planar [2][K_pad][rows_pad], natural K order
  int rows_pad, K_pad, Ko_pad, Ko, Ku, nocc, nu, nb, nrows;
  const double* w;       // this term's weights, natural order [K_pad]
  const double* dw;      // d weight / d energy [K_pad]
  double ct, pf;
  const BwdTile* tiles;
  double* grad;          // complex128 [nk][nb][nrows]
  double* part;          // [nparts][K_pad]
  // split GEMM only
  const __bf16* hs_u;    // Hu, Ho in operand tiles (h_tile_offset), blocks at h_off
  const __bf16* hs_o;
  const __bf16* psis;    // psi in operand tiles: 4 KiB groups [srows / 16][K_pad / 32], sites
                         // in 64-row slots (rows: K, contraction: site rows)
  int srows;
  int ntiles, per;       // tiles, and tiles per eighth of the grid
};

// Y = H psi for one site: rows p of H (64 per workgroup) x K columns (128 per workgroup),
// contracted over the site's points r' in chunks of 16, as a complex FP64 GEMM (cgemm64.h):
// lane l of matrix-core step s takes r' = 4 (l/16) + s, so both operands come from their
// natural layouts, H row-major (row stride npad) and psi planar [K][rows].
constexpr int BM = CG_BM, BN = CG_BN;
constexpr int BW_MB = CG_MB, BW_NB = CG_NB;

__global__ __launch_bounds__(256) void bwd_gemm_kernel(BwdParams P) {
  __shared__ __attribute__((aligned(1024))) unsigned char slot0[CG_STAGE];
  __shared__ __attribute__((aligned(1024))) unsigned char slot1[CG_STAGE];
  __shared__ double red[2][BN];
  const BwdTile tl = P.tiles[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / CG_WN, wn = wave % CG_WN;
  const bool occ = tl.k0 < P.Ko_pad;
  const size_t plane = (size_t)P.K_pad * P.rows_pad;
  // this wave loads plane (wave / 2), half (wave % 2) of every tile of a chunk
  const int pl = wave >> 1, hf = wave & 1;
  const double* hsrc = (pl == 0 ? (occ ? P.hu_re : P.ho_re) : (occ ? P.hu_im : P.ho_im)) + tl.h_off;
  const int lr = lane & 15, lg = lane >> 4;
  const double* asrc[CG_AT];
#pragma unroll
  for (int t = 0; t < CG_AT; ++t) {
    // rows past the block read its last row (their results are not stored)
    const int row = min(tl.r0 + 16 * t + lr, tl.npad - 1);
    asrc[t] = hsrc + (size_t)row * tl.npad + 4 * lg + 2 * hf;
  }
  const double* bsrc[CG_BT];
#pragma unroll
  for (int t = 0; t < CG_BT; ++t)
    bsrc[t] = P.psi + pl * plane + (size_t)(tl.k0 + 16 * t + lr) * P.rows_pad + tl.site_row0 +
              4 * lg + 2 * hf;
  f64x4 cr[BW_MB][BW_NB], ci[BW_MB][BW_NB];
#pragma unroll
  for (int i = 0; i < BW_MB; ++i)
#pragma unroll
    for (int j = 0; j < BW_NB; ++j) {
      cr[i][j] = f64x4{0, 0, 0, 0};
      ci[i][j] = f64x4{0, 0, 0, 0};
    }
  cgemm64_tile(asrc, bsrc, tl.npad / CG_KC, wave, lane, slot0, slot1, cr, ci);
  // epilogue: f64 accumulator element e of lane holds (row 4e + lane/16, col lane%16).  Per
  // accumulator block all loads are issued before the first use (entries outside the site or
  // in K padding read a valid address and store nothing).
  double colsum[BW_NB];
#pragma unroll
  for (int j = 0; j < BW_NB; ++j) {
    colsum[j] = 0.0;
    const int K = tl.k0 + (wn * BW_NB + j) * 16 + (lane & 15);
    int kp = -1, band = 0;
    if (occ && K < P.Ko) {
      kp = K / P.nocc;
      band = K - kp * P.nocc;
    } else if (!occ && K - P.Ko_pad < P.Ku) {
      const int q = K - P.Ko_pad;
      kp = q / P.nu;
      band = P.nocc + (q - kp * P.nu);
    }
    const double gw = 2.0 * P.pf * P.ct * P.w[K];
    const double ew = P.pf * P.ct * P.dw[K];
    const size_t gbase = (size_t)(max(kp, 0) * P.nb + band) * P.nrows;
#pragma unroll
    for (int i = 0; i < BW_MB; ++i) {
      bool ok[4];
      size_t gidx[4], o[4];
      double gre[4], gim[4], pre[4], pim[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = tl.r0 + (wm * BW_MB + i) * 16 + 4 * e + (lane >> 4);
        ok[e] = kp >= 0 && row < tl.ns;
        const int grow = tl.site_row0 + min(row, tl.ns - 1);
        gidx[e] = 2 * (gbase + grow);
        o[e] = (size_t)K * P.rows_pad + grow;
        gre[e] = P.grad[gidx[e]];
        gim[e] = P.grad[gidx[e] + 1];
        pre[e] = P.psi[o[e]];
        pim[e] = P.psi[plane + o[e]];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double yr = cr[i][j][e], yi = ci[i][j][e];
        if (ok[e]) {
          P.grad[gidx[e]] = gre[e] + gw * yr;
          P.grad[gidx[e] + 1] = gim[e] + gw * yi;
          colsum[j] += ew * (pre[e] * yr + pim[e] * yi);
        }
      }
    }
  }
  // reduce the energy partials over the tile's rows
#pragma unroll
  for (int j = 0; j < BW_NB; ++j) {
    double v = colsum[j];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    colsum[j] = v;
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < BW_NB; ++j) red[wm][(wn * BW_NB + j) * 16 + lane] = colsum[j];
  }
  __syncthreads();
  if (tid < BN) {
    double* p = P.part + (size_t)tl.part_row * P.K_pad + tl.k0 + tid;
    *p += red[0][tid] + red[1][tid];
  }
}

// The same product in split precision: Y = H psi with H = H_hi + H_lo and psi = psi_hi +
// psi_lo in bfloat16, each real product taken as hi*hi + hi*lo + lo*hi on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation.  Lane l of an instruction holds row (or
// column) l%32 and r' = 8 (l/32) + e, e = 0..7.  Both operands are stored in that order
// (h_tile_offset: 1 KiB per 32 rows x 16 r' x plane, planes of a piece adjacent, chunks of r'
// outermost), so every wave-wide direct-to-LDS load moves one contiguous KiB and every
// fragment read is a conflict-free 16-byte LDS read.  128 x 128 workgroup tiles (2 x 2 waves
// of 64 x 64), a four-slot ring, and the epilogue of the FP64 GEMM with Y converted to FP64.
// Workgroup b takes tile (b % 8) * per + b / 8, so the workgroups resident on one XCD run a
// contiguous stretch of the tile list, which the host orders in blocks of 4 row tiles x 8
// column tiles.
constexpr int SM = 128, SN = 128;
constexpr int S_AB = SM / 32, S_BB = SN / 32;     // 32-row (column) blocks per tile
constexpr int S_PIECES = (S_AB + S_BB) * 4;       // 1 KiB pieces per chunk: blocks x 4 planes
constexpr int S_STAGE = S_PIECES * 1024;
constexpr int S_LPW = S_PIECES / 4;               // loads per wave per chunk
constexpr int S_KEEP = 2 * S_LPW;                 // loads of chunks q+2, q+3 in flight at step q

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(unsigned int)))) unsigned int u32x4;

__global__ __launch_bounds__(256) void bwd_split_kernel(BwdParams P) {
  __shared__ __attribute__((aligned(1024))) unsigned char s0[S_STAGE];
  __shared__ __attribute__((aligned(1024))) unsigned char s1[S_STAGE];
  __shared__ __attribute__((aligned(1024))) unsigned char s2[S_STAGE];
  __shared__ __attribute__((aligned(1024))) unsigned char s3[S_STAGE];
  static_assert(S_STAGE == 64 * SM * 4, "a ring slot holds Y_re or Y_im of 64 K of the tile");
  const int ti = (blockIdx.x & 7) * P.per + (blockIdx.x >> 3);
  if (ti >= P.ntiles) return;
  const BwdTile tl = P.tiles[ti];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const bool occ = tl.k0 < P.Ko_pad;
  // wave w loads plane w of every block of a chunk: piece j = 4 t + w of the A blocks, then of
  // the B blocks
  const int lr = lane & 31, lh = lane >> 5;
  const int hb = tl.npad >> 5;    // 32-row blocks of the H block
  const __bf16* asrc[S_AB];
#pragma unroll
  for (int t = 0; t < S_AB; ++t) {
    // blocks past the H block read its last one (their results are not stored)
    const int rb = min((tl.r0 >> 5) + t, hb - 1);
    asrc[t] = (occ ? P.hs_u : P.hs_o) + tl.h_off + ((size_t)(4 * rb + wave) << 9) + lane * 8;
  }
  const size_t a_chunk = (size_t)hb << 11;
  const __bf16* bsrc[S_BB];
  const size_t b_chunk = (size_t)(P.K_pad >> 5) << 11;
#pragma unroll
  for (int t = 0; t < S_BB; ++t)
    bsrc[t] = P.psis + (size_t)(tl.srow0 >> 4) * b_chunk +
              ((size_t)(4 * ((tl.k0 >> 5) + t) + wave) << 9) + lane * 8;
  const size_t plane = (size_t)P.K_pad * P.rows_pad;
  const int nch = tl.npad / 16;   // a multiple of 4
  auto issue = [&](int c, unsigned char* dst) {
    c = min(c, nch - 1);          // past the end: the last chunk again, never read
#pragma unroll
    for (int t = 0; t < S_AB; ++t)
      __builtin_amdgcn_global_load_lds(
          (const void __attribute__((address_space(1)))*)(asrc[t] + c * a_chunk),
          (void __attribute__((address_space(3)))*)(dst + (4 * t + wave) * 1024), 16, 0, 0);
#pragma unroll
    for (int t = 0; t < S_BB; ++t)
      __builtin_amdgcn_global_load_lds(
          (const void __attribute__((address_space(1)))*)(bsrc[t] + c * b_chunk),
          (void __attribute__((address_space(3)))*)(dst + (4 * (S_AB + t) + wave) * 1024), 16, 0,
          0);
  };
  struct Frag {
    bf16x8 a[2][4], b[2][4];   // [block][plane]
  };
  auto load = [&](const unsigned char* sl, Frag& f) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        f.a[i][p] = *(const bf16x8*)(sl + (4 * (2 * wm + i) + p) * 1024 + lane * 16);
        f.b[i][p] = *(const bf16x8*)(sl + (4 * (S_AB + 2 * wn + i) + p) * 1024 + lane * 16);
      }
  };
  f32x16 yr[2][2], yi[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        yr[i][j][e] = 0.f;
        yi[i][j][e] = 0.f;
      }
  // Yr += Hr psi_r - Hi psi_i, Yi += Hr psi_i + Hi psi_r (planes 0, 1 = re hi, lo; 2, 3 = im),
  // each real product as hi*hi + hi*lo + lo*hi.  Products go in the outer loop, so that the
  // four blocks' accumulators take turns and consecutive instructions never depend on each
  // other.
  auto mma = [&](const Frag& f) {
    const u32x4 m = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    bf16x8 ni[2][2];   // -Hi hi, -Hi lo per block
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ni[i][0] = (bf16x8)((u32x4)f.a[i][2] ^ m);
      ni[i][1] = (bf16x8)((u32x4)f.a[i][3] ^ m);
    }
    // {A plane (4, 5: -Hi hi, -Hi lo), B plane, target (0: Yr, 1: Yi)}
    constexpr int prod[12][3] = {{0, 0, 0}, {0, 2, 1}, {0, 1, 0}, {0, 3, 1},
                                 {1, 0, 0}, {1, 2, 1}, {4, 2, 0}, {2, 0, 1},
                                 {4, 3, 0}, {2, 1, 1}, {5, 2, 0}, {3, 0, 1}};
#pragma unroll
    for (int p = 0; p < 12; ++p)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const bf16x8 a = prod[p][0] >= 4 ? ni[i][prod[p][0] - 4] : f.a[i][prod[p][0]];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          f32x16& acc = prod[p][2] ? yi[i][j] : yr[i][j];
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, f.b[j][prod[p][1]], acc, 0, 0, 0);
        }
      }
  };
  constexpr int kMFMA = 0x008, kVMEM = 0x010, kDSREAD = 0x100;
  constexpr int NMF = 48, NDS = 16, NVM = S_LPW;
  constexpr int R = (NMF - NDS) / (NVM + 1), REST = NMF - NDS - R * NVM;
  auto sched = [] {
    sched_pairs<NDS, kMFMA, 1, kDSREAD, 1>();
    sched_pairs<NVM, kMFMA, R, kVMEM, 1>();
    __builtin_amdgcn_sched_group_barrier(kMFMA, REST, 0);
  };
  // step q: chunk q+1 has landed (the loads of q+2 and q+3 may be in flight) and every wave
  // has read chunk q's slot out; read chunk q+1's fragments, load chunk q+4 into chunk q's
  // slot, matrix-core instructions of chunk q
  Frag fa, fb;
  int q = 0;
  auto step = [&](const unsigned char* next, unsigned char* mine, Frag& cur, Frag& nxt) {
    ring_barrier<S_KEEP>();
    load(next, nxt);
    issue(q + 4, mine);
    mma(cur);
    sched();
    __builtin_amdgcn_sched_barrier(0);
    ++q;
  };
  issue(0, s0);
  issue(1, s1);
  issue(2, s2);
  issue(3, s3);
  ring_barrier<3 * S_LPW>();
  load(s0, fa);
  while (q < nch) {
    step(s1, s0, fa, fb);
    step(s2, s1, fb, fa);
    step(s3, s2, fa, fb);
    step(s0, s3, fb, fa);
  }
  ring_barrier<0>();
  // epilogue.  Element e of a lane's 32 x 32 accumulator block is (row 8 (e/4) + 4 (lane/32) +
  // e%4, column lane%32): the lanes of an instruction span 32 K, whose gradient and orbital
  // rows lie far apart in memory.  So Y goes through the ring's LDS first, Y_re in s0 (K 0..63
  // of the tile) and s1 (K 64..127), Y_im in s2 and s3, each [K][128 rows] in FP32 with the row
  // index XOR-ed with K % 32 (the accumulator writes then fall in distinct banks).  Then wave w
  // takes K = w, w + 4, ..., eight at a time, with the lanes along the tile's rows: the FP64
  // gradient and the orbitals are read and written along contiguous site rows, and each K's
  // energy partial is a sum within one wave.
  {
    float* yre_s = (float*)(wn ? s1 : s0);
    float* yim_s = (float*)(wn ? s3 : s2);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int row = wm * 64 + 32 * i + 8 * (e >> 2) + 4 * lh + (e & 3);
          const int o = (32 * j + lr) * SM + (row ^ lr);
          yre_s[o] = yr[i][j][e];
          yim_s[o] = yi[i][j][e];
        }
  }
  __syncthreads();
  constexpr int KB = 8;   // K per batch: every load of a batch is issued before the first use
  for (int kb = 0; kb < SN / 4; kb += KB) {
    int kk[KB], kpv[KB], bandv[KB];
    double gre[KB][2], gim[KB][2], pre[KB][2], pim[KB][2];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      kk[u] = wave + 4 * (kb + u);
      const int K = tl.k0 + kk[u];
      int kp = -1, band = 0;
      if (occ && K < P.Ko) {
        kp = K / P.nocc;
        band = K - kp * P.nocc;
      } else if (!occ && K - P.Ko_pad < P.Ku) {
        const int qq = K - P.Ko_pad;
        kp = qq / P.nu;
        band = P.nocc + (qq - kp * P.nu);
      }
      kpv[u] = kp;
      bandv[u] = band;
      const size_t gbase = (size_t)(max(kp, 0) * P.nb + band) * P.nrows;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // rows past the site read its last row (their results are not stored)
        const int grow = tl.site_row0 + min(tl.r0 + lane + 64 * h, tl.ns - 1);
        const double2 g = *(const double2*)(P.grad + 2 * (gbase + grow));
        const size_t o = (size_t)K * P.rows_pad + grow;
        gre[u][h] = g.x;
        gim[u][h] = g.y;
        pre[u][h] = P.psi[o];
        pim[u][h] = P.psi[plane + o];
      }
    }
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      if (kpv[u] < 0) continue;   // K padding (wave-uniform)
      const int K = tl.k0 + kk[u];
      const double gw = 2.0 * P.pf * P.ct * P.w[K];
      const double ew = P.pf * P.ct * P.dw[K];
      const size_t gbase = (size_t)(kpv[u] * P.nb + bandv[u]) * P.nrows;
      const int kl = kk[u] & 63;
      const float* yre_s = (const float*)(kk[u] < 64 ? s0 : s1);
      const float* yim_s = (const float*)(kk[u] < 64 ? s2 : s3);
      double sum = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int row = lane + 64 * h;
        if (tl.r0 + row < tl.ns) {
          const int o = kl * SM + (row ^ (kl & 31));
          const double vr = (double)yre_s[o], vi = (double)yim_s[o];
          const int grow = tl.site_row0 + tl.r0 + row;
          *(double2*)(P.grad + 2 * (gbase + grow)) =
              double2{gre[u][h] + gw * vr, gim[u][h] + gw * vi};
          sum += ew * (pre[u][h] * vr + pim[u][h] * vi);
        }
      }
      for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
      if (lane == 0) P.part[(size_t)tl.part_row * P.K_pad + K] += sum;
    }
  }
}

// psi planes [2][K_pad][rows_pad] (FP64, compact site rows) -> the split GEMM's B operand:
// bfloat16 hi/lo of re and im in operand tiles with K as the row and the site row (in 64-row
// slots, rowmap[slot row] = compact row or -1) as the contraction index
__global__ void split_psi_kernel(const double* psi, int rows_pad, int K_pad, const int* rowmap,
                                 int srows, __bf16* out) {
  const long long n = (long long)K_pad * srows;
  const size_t pin = (size_t)K_pad * rows_pad;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int K = (int)(i / srows), sr = (int)(i - (long long)K * srows);
    const int r = rowmap[sr];
    const double re = r >= 0 ? psi[(size_t)K * rows_pad + r] : 0.0;
    const double im = r >= 0 ? psi[pin + (size_t)K * rows_pad + r] : 0.0;
    const __bf16 rh = (__bf16)(float)re, ih = (__bf16)(float)im;
    const long long o = h_tile_offset(K, sr, K_pad);
    out[o] = rh;
    out[o + 512] = (__bf16)(float)(re - (double)(float)rh);
    out[o + 1024] = ih;
    out[o + 1536] = (__bf16)(float)(im - (double)(float)ih);
  }
}

// lam = (A + A^T) / 2 per site, from the caller's n x n blocks (offsets blk_off) into blocks
// with row stride npad (offsets pblk_off); the padding rows and columns are zero
// symmetric part of each site block of lam into the padded layout, and the antisymmetric part
// too where out_a is given
__global__ void symmetrise_kernel(const double* lam, const long long* blk_off,
                                  const long long* pblk_off, const int* blk_n, int nsites,
                                  double* out, double* out_a) {
  const int s = blockIdx.y;
  if (s >= nsites) return;
  const int n = blk_n[s], np = (n + kAdjAlign - 1) / kAdjAlign * kAdjAlign;
  const double* a = lam + blk_off[s];
  double* o = out + pblk_off[s];
  for (long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x; it < (long long)np * np;
       it += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(it / np), c = (int)(it % np);
    const bool in = r < n && c < n;
    const double x = in ? a[(long long)r * n + c] : 0.0, y = in ? a[(long long)c * n + r] : 0.0;
    o[it] = 0.5 * (x + y);
    if (out_a) out_a[pblk_off[s] + it] = 0.5 * (x - y);
  }
}

__global__ void reduce_energy_kernel(const double* part, int nparts, int K_pad, int Ko, int Ko_pad,
                                     int Ku, int nocc, int nu, int nb, double* dE) {
  const int K = blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= K_pad) return;
  int kp = -1, band = 0;
  if (K < Ko) {
    kp = K / nocc;
    band = K - kp * nocc;
  } else if (K >= Ko_pad && K - Ko_pad < Ku) {
    const int q = K - Ko_pad;
    kp = q / nu;
    band = nocc + (q - kp * nu);
  }
  if (kp < 0) return;
  double s = 0;
  for (int p = 0; p < nparts; ++p) s += part[(size_t)p * K_pad + K];
  dE[kp * nb + band] = s;
}

hipError_t ensure(lrs_ctx* ctx, DevBuf& b, size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  if (b.p && b.bytes >= bytes) return hipSuccess;
  if (b.p) {
    (void)hipFree(b.p);
    ctx->bytes_in_use -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  if (ctx->max_bytes && ctx->bytes_in_use + bytes > ctx->max_bytes) return hipErrorOutOfMemory;
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    b.p = nullptr;
    return hipErrorOutOfMemory;
  }
  b.bytes = bytes;
  ctx->bytes_in_use += bytes;
  return hipSuccess;
}

}  // namespace

hipError_t launch_chi0_backward(lrs_ctx* ctx, int prec, const double* dL_dchi0, double* dL_dE,
                                double* dL_dpsi) {
  hipStream_t st = ctx->stream;
  // the Green's functions in `prec` (F16F8: the 128 x 128 tile, whose site block has more
  // tiles to spread over the workgroups than the 128 x 192 one); the products with psi in
  // split bfloat16 for both reduced precisions, else FP64
  const bool split = prec == LRS_BF16X2 || prec == LRS_F16F8;
  const int gvar = prec == LRS_F16F8 ? 1 : 0;
  // real orbitals (two per operand slot): the products with psi run over the 2 K_pad orbitals
  // in their own order, with zero imaginary parts, and H comes from the kept Green's functions
  const bool real = ctx->real_mode;
  const int Kb = real ? 2 * ctx->K_pad : ctx->K_pad;
  const int Kob = real ? 2 * ctx->Ko_pad : ctx->Ko_pad;
  if (real && !(prec == LRS_F16F8 && ctx->g_keep_prec == LRS_F16F8)) return hipErrorInvalidValue;
  // operands: site rows and site columns of the precision, k-major orbitals (FP64, and split)
  if (ensure_site_tiles_for(ctx, prec) != LRS_OK) return hipErrorOutOfMemory;
  Plan* plan = nullptr;
  if (plan_for(ctx, -1, LRS_COLS_SITE, prec, gvar, 1, &plan) != LRS_OK) return hipErrorOutOfMemory;
  // (the k-major orbitals and their split copy depend on the orbitals and sites only: built
  // once, dropped with the sites)
  hipError_t e = hipSuccess;
  if (!ctx->psi_kmajor_ok) {
    e = ensure(ctx, ctx->psi_site_f64, (size_t)2 * Kb * ctx->rows_pad * 8);
    if (e != hipSuccess) return e;
    e = launch_derive_site_kmajor((const double*)ctx->site_f64.p, ctx->rows_pad, ctx->K_pad,
                                  real ? 1 : 0, (double*)ctx->psi_site_f64.p, st);
    if (e != hipSuccess) return e;
    ctx->psi_kmajor_ok = true;
  }

  // site blocks (the caller's n x n layout, and the padded one of the H arrays), the split
  // orbital rows (64-row slot per site) and the GEMM tile list
  const int S = ctx->nsites;
  const int tm = split ? SM : BM, tn = split ? SN : BN;
  std::vector<long long> blk_off(S), pblk_off(S);
  std::vector<int> blk_n(S), rowmap;
  std::vector<BwdTile> tiles;
  long long tot = 0, ptot = 0;
  int nparts = 0, srows = 0;
  if (Kb % tn) return hipErrorInvalidValue;
  const int nkt = Kb / tn;
  for (int s = 0; s < S; ++s) {
    const int n = ctx->site_off[s + 1] - ctx->site_off[s];
    const int np = site_block_ld(n, 1);
    blk_off[s] = tot;
    pblk_off[s] = ptot;
    blk_n[s] = n;
    const int nrt = (n + tm - 1) / tm;
    auto add = [&](int rt, int kt) {
      // (the split H holds four planes per block element)
      tiles.push_back(BwdTile{ctx->site_off[s], rt * tm, n, kt * tn, split ? 4 * ptot : ptot,
                              nparts + rt, np, srows});
    };
    if (split) {
      // blocks of 4 row tiles x 8 column tiles
      for (int r0 = 0; r0 < nrt; r0 += 4)
        for (int k0 = 0; k0 < nkt; k0 += 8)
          for (int r = r0; r < std::min(r0 + 4, nrt); ++r)
            for (int k = k0; k < std::min(k0 + 8, nkt); ++k) add(r, k);
      for (int i = 0; i < np; ++i) rowmap.push_back(i < n ? ctx->site_off[s] + i : -1);
      srows += np;
    } else {
      for (int r = 0; r < nrt; ++r)
        for (int k = 0; k < nkt; ++k) add(r, k);
    }
    nparts += nrt;
    tot += (long long)n * n;
    ptot += (long long)np * np;
  }
  const int T = ctx->quad.nterms;
  const size_t Kp = Kb;
  // workspace: lam | H (FP64: hu_re | hu_im | ho_re | ho_im; split: hs_u | hs_o, four bfloat16
  // planes each) over the padded blocks | part | w | dw | tiles | blk_off | pblk_off | blk_n |
  // rowmap (split)
  const bool odd = !ctx->quad.ci.empty();   // complex term coefficients
  const size_t hbytes = split ? (size_t)16 * ptot : (size_t)32 * ptot;
  size_t bytes = (size_t)ptot * 8 * (odd ? 2 : 1) + hbytes + (size_t)nparts * Kp * 8 +
                 2 * (size_t)T * Kp * 8 +
                 tiles.size() * sizeof(BwdTile) + S * 16 + S * 4 + rowmap.size() * 4 + 4096;
  e = ensure(ctx, ctx->adj_work, bytes);
  if (e != hipSuccess) return e;
  if (split) {
    const void* had = ctx->psi_site_bf16.p;
    e = ensure(ctx, ctx->psi_site_bf16, (size_t)8 * Kp * srows);
    if (e != hipSuccess) return e;
    if (ctx->psi_site_bf16.p != had) ctx->psi_split_ok = false;
  }
  char* p = (char*)ctx->adj_work.p;
  auto take = [&](size_t b) {
    char* q = p;
    p += (b + 255) / 256 * 256;
    return q;
  };
  double* lam = (double*)take(ptot * 8);
  double* lam_a = odd ? (double*)take(ptot * 8) : nullptr;
  char* hbuf = take(hbytes);
  double* part = (double*)take((size_t)nparts * Kp * 8);
  double* wn = (double*)take((size_t)T * Kp * 8);
  double* dwn = (double*)take((size_t)T * Kp * 8);
  BwdTile* dtiles = (BwdTile*)take(tiles.size() * sizeof(BwdTile));
  long long* dblk_off = (long long*)take(S * 8);
  long long* dpblk_off = (long long*)take(S * 8);
  int* dblk_n = (int*)take(S * 4);
  int* drowmap = (int*)take(rowmap.size() * 4);
  if ((size_t)(p - (char*)ctx->adj_work.p) > ctx->adj_work.bytes) return hipErrorOutOfMemory;
  double* hu_re = split ? nullptr : (double*)hbuf;
  double* hu_im = split ? nullptr : hu_re + ptot;
  double* ho_re = split ? nullptr : hu_re + 2 * ptot;
  double* ho_im = split ? nullptr : hu_re + 3 * ptot;
  __bf16* hs_u = split ? (__bf16*)hbuf : nullptr;
  __bf16* hs_o = split ? hs_u + 4 * ptot : nullptr;

  const std::vector<double>& wsrc = real ? ctx->quad.w_orb : ctx->quad.w;
  const std::vector<double>& dwsrc = real ? ctx->quad.dw_orb : ctx->quad.dw;
  if (wsrc.size() < (size_t)T * Kp || dwsrc.size() < (size_t)T * Kp) return hipErrorInvalidValue;
  if ((e = hipMemcpyAsync(wn, wsrc.data(), (size_t)T * Kp * 8, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(dwn, dwsrc.data(), (size_t)T * Kp * 8, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(dtiles, tiles.data(), tiles.size() * sizeof(BwdTile), hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(dblk_off, blk_off.data(), S * 8, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(dpblk_off, pblk_off.data(), S * 8, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(dblk_n, blk_n.data(), S * 4, hipMemcpyHostToDevice, st)))
    return e;
  if (split && !ctx->psi_split_ok) {
    if ((e = hipMemcpyAsync(drowmap, rowmap.data(), rowmap.size() * 4, hipMemcpyHostToDevice, st)))
      return e;
    hipLaunchKernelGGL(split_psi_kernel, dim3(4096), dim3(256), 0, st,
                       (const double*)ctx->psi_site_f64.p, ctx->rows_pad, Kb, drowmap,
                       srows, (__bf16*)ctx->psi_site_bf16.p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ctx->psi_split_ok = true;
  }
  hipLaunchKernelGGL(symmetrise_kernel, dim3(256, S), dim3(256), 0, st, dL_dchi0, dblk_off,
                     dpblk_off, dblk_n, S, lam, lam_a);
  // the adjoint Green's-function launches write the blocks' valid entries only: the padding
  // of the H arrays must read as zero in the contraction
  if ((e = launch_fill_zero(hbuf, hbytes, st)) ||
      (e = launch_fill_zero(part, (size_t)nparts * Kp * 8, st)) ||
      (e = launch_fill_zero(dL_dpsi, (size_t)2 * ctx->nk * ctx->nb * ctx->nrows * 8, st)))
    return e;

  BwdParams B;
  B.hu_re = hu_re;
  B.hu_im = hu_im;
  B.ho_re = ho_re;
  B.ho_im = ho_im;
  B.psi = (const double*)ctx->psi_site_f64.p;
  B.rows_pad = ctx->rows_pad;
  B.K_pad = Kb;
  B.Ko_pad = Kob;
  B.Ko = ctx->Ko;
  B.Ku = ctx->Ku;
  B.nocc = ctx->nocc;
  B.nu = ctx->nu;
  B.nb = ctx->nb;
  B.nrows = ctx->nrows;
  B.pf = -2.0 * ctx->spin / ((double)ctx->nk * ctx->nk);
  B.tiles = dtiles;
  B.grad = dL_dpsi;
  B.part = part;
  B.hs_u = hs_u;
  B.hs_o = hs_o;
  B.psis = split ? (const __bf16*)ctx->psi_site_bf16.p : nullptr;
  B.srows = srows;
  B.ntiles = (int)tiles.size();
  B.per = (B.ntiles + 7) / 8;
  const int chunk = chunk_of(prec);
  const double g_scale = is_f16(prec) ? (double)ctx->site_scale_f16 * ctx->site_scale_f16 : 1.0;
  // the Green's functions an F16F8 or BF16X2 launch over every site block kept (same
  // quadrature, sites and orbitals; any change of those drops them): H from them instead of
  // recomputing G
  const size_t kelem = prec == LRS_FP64 ? 16 : 8;
  const bool kept = (prec == LRS_F16F8 || prec == LRS_BF16X2 || prec == LRS_FP64) &&
                    ctx->g_keep_prec == prec && ctx->g_keep.p &&
                    ctx->g_keep.bytes >= (size_t)2 * T * tot * kelem;
  if (real && !kept) return hipErrorInvalidValue;    // (the entry point checks this first)
  for (int t = 0; t < T; ++t) {
    if (kept) {
      const char* ko = (const char*)ctx->g_keep.p + (size_t)t * tot * kelem;
      const char* ku = ko + (size_t)T * tot * kelem;
      const double ac = odd ? ctx->quad.c[t] : 0.0, as = odd ? ctx->quad.ci[t] : 0.0;
      if (split)
        e = launch_h_from_kept(ko, ku, S, dblk_off, dpblk_off, dblk_n, blk_n.data(), lam, lam_a,
                               ac, as, hs_u, hs_o, st);
      else
        e = launch_h_from_kept_f64(ko, ku, S, dblk_off, dpblk_off, dblk_n, lam, lam_a, ac, as,
                                   hu_re, hu_im, ho_re, ho_im, st);
      if (e != hipSuccess) return e;
    }
    for (const Batch& bt : plan->batches) {
      if (kept || bt.ntiles == 0) continue;
      const void* a_op = nullptr;
      // (LRS_ESTATE: a buffer that captured graphs read would have to be replaced)
      lrs_status ls = ensure_site_operand(ctx, prec, bt, t, 1, &a_op);
      if (ls == LRS_OK) ls = ensure_park(ctx, prec, gvar, bt.grid);
      if (ls != LRS_OK) return ls == LRS_ESTATE ? hipErrorIllegalState : hipErrorOutOfMemory;
      e = launch_green_adjoint(prec, bt.grid, a_op, bt.nrb, ctx->site_tiles[prec].p,
                               ctx->site_cols_pad / 16, ctx->K_pad / chunk,
                               (const double*)ctx->c_dev.p + t, ctx->Ko_pad / chunk,
                               (const TileDesc*)plan->tiles.p + bt.tile0, bt.ntiles, lam, lam_a,
                               odd ? ctx->quad.c[t] : 0.0, odd ? ctx->quad.ci[t] : 0.0, hu_re,
                               hu_im, ho_re, ho_im, hs_u, hs_o, ctx->park.p, st);
      if (e != hipSuccess) return e;
    }
    B.w = wn + (size_t)t * Kp;
    B.dw = dwn + (size_t)t * Kp;
    // (complex coefficients are inside H; fp16-prescaled operands scale each G, and so H, by
    // the square of the site prescale, a power of two taken out here)
    B.ct = (odd ? 1.0 : ctx->quad.c[t]) / g_scale;
    if (split)
      hipLaunchKernelGGL(bwd_split_kernel, dim3((unsigned)(8 * B.per)), dim3(256), 0, st, B);
    else
      hipLaunchKernelGGL(bwd_gemm_kernel, dim3((unsigned)tiles.size()), dim3(256), 0, st, B);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(reduce_energy_kernel, dim3((Kb + 255) / 256), dim3(256), 0, st, part,
                     nparts, Kb, ctx->Ko, Kob, ctx->Ku, ctx->nocc, ctx->nu, ctx->nb,
                     dL_dE);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // host tables are freed on return
  return e;
}

}  // namespace lrs
