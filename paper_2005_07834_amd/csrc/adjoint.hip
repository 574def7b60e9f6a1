// Adjoint of chi0 on site x site blocks (FP64).
//
// With P_f = -2 s / N_k^2, Lambda = dL/dchi0 (symmetrised: chi0 on a square block is symmetric)
// and per term l the weighted Green's functions G_o^l, G_u^l of the forward pass,
//   dL/dpsi_K (K occupied)   = 2 P_f sum_l c_l alpha_l(K) [ (Lambda o conj(G_u^l)) psi_K ]
//   dL/dpsi_K (K unoccupied) = 2 P_f sum_l c_l beta_l(K)  [ (Lambda o conj(G_o^l)) psi_K ]
//   dL/de_K = P_f sum_l c_l (d weight_l(K)/d e_K) Re[ psi_K^H (Lambda o conj(G^l)) psi_K ]
// (complex gradients as dL/dRe + i dL/dIm; mu and the nodes held fixed).  Each term's G's are
// recomputed on the matrix cores (the chi0 kernel in its adjoint mode writes
// Lambda o conj(G) directly); the products with psi run as a complex FP64 MFMA GEMM whose
// epilogue accumulates the orbital gradient and per-row-tile energy partials.  Every output
// element has one owner per launch and launches are ordered, so results are bitwise
// reproducible.
#include <hip/hip_runtime.h>

#include <vector>

#include "lrs_internal.h"

namespace lrs {
namespace {

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double f64x4;

struct BwdTile {
  int site_row0;       // first global row of the site
  int r0;              // first local row of this tile
  int ns;              // points of the site
  int k0;              // first K column of this tile
  long long h_off;     // offset of the site's block in the H arrays
  int part_row;        // row-tile index for the energy partials
  int pad;
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
};

constexpr int BM = 64, BN = 64, BK = 16;

__global__ __launch_bounds__(256) void bwd_gemm_kernel(BwdParams P) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[(BM / 16 + BN / 16) * kTileBytes];
  __shared__ double red[2][BN];
  unsigned char* la = lds;
  unsigned char* lb = lds + (BM / 16) * kTileBytes;
  const BwdTile tl = P.tiles[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  const bool occ = tl.k0 < P.Ko_pad;
  const double* hre = (occ ? P.hu_re : P.ho_re) + tl.h_off;
  const double* him = (occ ? P.hu_im : P.ho_im) + tl.h_off;
  const size_t plane = (size_t)P.K_pad * P.rows_pad;
  f64x4 cr[2][2], ci[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = f64x4{0, 0, 0, 0};
      ci[i][j] = f64x4{0, 0, 0, 0};
    }
  for (int kc = 0; kc < tl.ns; kc += BK) {
    __syncthreads();
    for (int it = tid; it < BM * BK; it += 256) {
      const int m = it / BK, kk = it % BK;
      const int row = tl.r0 + m, k = kc + kk;
      double ar = 0, ai = 0;
      if (row < tl.ns && k < tl.ns) {
        ar = hre[(long long)row * tl.ns + k];
        ai = him[(long long)row * tl.ns + k];
      }
      const int ln = (kk & 3) * 16 + (m & 15), s = kk >> 2;
      double* dst = (double*)(la + (m >> 4) * kTileBytes);
      dst[ln * 4 + s] = ar;
      dst[256 + ln * 4 + s] = ai;
    }
    for (int it = tid; it < BN * BK; it += 256) {
      const int n = it / BK, kk = it % BK;
      const int k = kc + kk;
      double br = 0, bi = 0;
      if (k < tl.ns) {
        const size_t o = (size_t)(tl.k0 + n) * P.rows_pad + tl.site_row0 + k;
        br = P.psi[o];
        bi = P.psi[plane + o];
      }
      const int ln = (kk & 3) * 16 + (n & 15), s = kk >> 2;
      double* dst = (double*)(lb + (n >> 4) * kTileBytes);
      dst[ln * 4 + s] = br;
      dst[256 + ln * 4 + s] = bi;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const double* a = (const double*)(la + (wm * 2 + i) * kTileBytes);
        ar[i] = a[lane * 4 + s];
        ai[i] = a[256 + lane * 4 + s];
        const double* b = (const double*)(lb + (wn * 2 + i) * kTileBytes);
        br[i] = b[lane * 4 + s];
        bi[i] = b[256 + lane * 4 + s];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cr[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bi[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], ci[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], ci[i][j], 0, 0, 0);
        }
    }
  }
  // epilogue: f64 accumulator element e of lane holds (row 4e + lane/16, col lane%16)
  double colsum[2] = {0.0, 0.0};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int K = tl.k0 + (wn * 2 + j) * 16 + (lane & 15);
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
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = tl.r0 + (wm * 2 + i) * 16 + 4 * e + (lane >> 4);
        if (kp < 0 || row >= tl.ns) continue;
        const int grow = tl.site_row0 + row;
        const double yr = cr[i][j][e], yi = ci[i][j][e];
        double* g = P.grad + 2 * ((size_t)(kp * P.nb + band) * P.nrows + grow);
        g[0] += gw * yr;
        g[1] += gw * yi;
        const size_t o = (size_t)K * P.rows_pad + grow;
        colsum[j] += ew * (P.psi[o] * yr + P.psi[plane + o] * yi);
      }
  }
  // reduce the energy partials over the tile's rows
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    double v = colsum[j];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    colsum[j] = v;
  }
  if (lane < 16) {
    red[wm][(wn * 2 + 0) * 16 + lane] = colsum[0];
    red[wm][(wn * 2 + 1) * 16 + lane] = colsum[1];
  }
  __syncthreads();
  if (tid < BN) {
    double* p = P.part + (size_t)tl.part_row * P.K_pad + tl.k0 + tid;
    *p += red[0][tid] + red[1][tid];
  }
}

__global__ void symmetrise_kernel(const double* lam, const long long* blk_off, const int* blk_n,
                                  int nsites, double* out) {
  const int s = blockIdx.y;
  if (s >= nsites) return;
  const int n = blk_n[s];
  const double* a = lam + blk_off[s];
  double* o = out + blk_off[s];
  for (long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x; it < (long long)n * n;
       it += (long long)gridDim.x * blockDim.x) {
    const int r = (int)(it / n), c = (int)(it % n);
    o[it] = 0.5 * (a[it] + a[(long long)c * n + r]);
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

hipError_t launch_chi0_backward(lrs_ctx* ctx, const double* dL_dchi0, double* dL_dE,
                                double* dL_dpsi) {
  hipStream_t st = ctx->stream;
  // operands: site rows (FP64), site columns (FP64 tiles), k-major orbitals
  if (ensure_site_tiles_for(ctx, LRS_FP64) != LRS_OK) return hipErrorOutOfMemory;
  Plan* plan = nullptr;
  if (plan_for(ctx, -1, LRS_COLS_SITE, LRS_FP64, 0, 1, &plan) != LRS_OK) return hipErrorOutOfMemory;
  hipError_t e = ensure(ctx, ctx->psi_site_f64, (size_t)2 * ctx->K_pad * ctx->rows_pad * 8);
  if (e != hipSuccess) return e;
  e = launch_derive_site_kmajor((const double*)ctx->site_f64.p, ctx->rows_pad, ctx->K_pad,
                                (double*)ctx->psi_site_f64.p, st);
  if (e != hipSuccess) return e;

  // site blocks and the GEMM tile list
  const int S = ctx->nsites;
  std::vector<long long> blk_off(S);
  std::vector<int> blk_n(S);
  std::vector<BwdTile> tiles;
  long long tot = 0;
  int nparts = 0;
  for (int s = 0; s < S; ++s) {
    const int n = ctx->site_off[s + 1] - ctx->site_off[s];
    blk_off[s] = tot;
    blk_n[s] = n;
    for (int r0 = 0; r0 < n; r0 += BM) {
      for (int k0 = 0; k0 < ctx->K_pad; k0 += BN)
        tiles.push_back(BwdTile{ctx->site_off[s], r0, n, k0, tot, nparts, 0});
      ++nparts;
    }
    tot += (long long)n * n;
  }
  const int T = ctx->quad.nterms;
  const size_t Kp = ctx->K_pad;
  // workspace: lam | hu_re | hu_im | ho_re | ho_im | part | w | dw | tiles | blk_off | blk_n
  size_t bytes = (size_t)5 * tot * 8 + (size_t)nparts * Kp * 8 + 2 * (size_t)T * Kp * 8 +
                 tiles.size() * sizeof(BwdTile) + S * 8 + S * 4 + 4096;
  e = ensure(ctx, ctx->adj_work, bytes);
  if (e != hipSuccess) return e;
  char* p = (char*)ctx->adj_work.p;
  auto take = [&](size_t b) {
    char* q = p;
    p += (b + 255) / 256 * 256;
    return q;
  };
  double* lam = (double*)take(tot * 8);
  double* hu_re = (double*)take(tot * 8);
  double* hu_im = (double*)take(tot * 8);
  double* ho_re = (double*)take(tot * 8);
  double* ho_im = (double*)take(tot * 8);
  double* part = (double*)take((size_t)nparts * Kp * 8);
  double* wn = (double*)take((size_t)T * Kp * 8);
  double* dwn = (double*)take((size_t)T * Kp * 8);
  BwdTile* dtiles = (BwdTile*)take(tiles.size() * sizeof(BwdTile));
  long long* dblk_off = (long long*)take(S * 8);
  int* dblk_n = (int*)take(S * 4);
  if ((size_t)(p - (char*)ctx->adj_work.p) > ctx->adj_work.bytes) return hipErrorOutOfMemory;

  if ((e = hipMemcpyAsync(wn, ctx->quad.w.data(), (size_t)T * Kp * 8, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(dwn, ctx->quad.dw.data(), (size_t)T * Kp * 8, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(dtiles, tiles.data(), tiles.size() * sizeof(BwdTile), hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(dblk_off, blk_off.data(), S * 8, hipMemcpyHostToDevice, st)) ||
      (e = hipMemcpyAsync(dblk_n, blk_n.data(), S * 4, hipMemcpyHostToDevice, st)))
    return e;
  hipLaunchKernelGGL(symmetrise_kernel, dim3(256, S), dim3(256), 0, st, dL_dchi0, dblk_off, dblk_n,
                     S, lam);
  if ((e = launch_fill_zero(part, (size_t)nparts * Kp * 8, st)) ||
      (e = launch_fill_zero(dL_dpsi, (size_t)2 * ctx->nk * ctx->nb * ctx->nrows * 8, st)))
    return e;

  BwdParams B;
  B.hu_re = hu_re;
  B.hu_im = hu_im;
  B.ho_re = ho_re;
  B.ho_im = ho_im;
  B.psi = (const double*)ctx->psi_site_f64.p;
  B.rows_pad = ctx->rows_pad;
  B.K_pad = ctx->K_pad;
  B.Ko_pad = ctx->Ko_pad;
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
  for (int t = 0; t < T; ++t) {
    for (const Batch& bt : plan->batches) {
      if (bt.ntiles == 0) continue;
      if (ensure_site_operand(ctx, LRS_FP64, bt, t, 1) != LRS_OK) return hipErrorOutOfMemory;
      if (ensure_park(ctx, LRS_FP64, 0, bt.grid) != LRS_OK) return hipErrorOutOfMemory;
      e = launch_green_adjoint(bt.grid, ctx->a_tiles.p, bt.nrb, ctx->site_tiles[LRS_FP64].p,
                               ctx->site_cols_pad / 16, ctx->K_pad / kChunkF64, (const double*)ctx->c_dev.p + t,
                               ctx->Ko_pad / kChunkF64, (const TileDesc*)plan->tiles.p + bt.tile0,
                               bt.ntiles, lam, hu_re, hu_im, ho_re, ho_im, ctx->park.p, st);
      if (e != hipSuccess) return e;
    }
    B.w = wn + (size_t)t * Kp;
    B.dw = dwn + (size_t)t * Kp;
    B.ct = ctx->quad.c[t];
    hipLaunchKernelGGL(bwd_gemm_kernel, dim3((unsigned)tiles.size()), dim3(256), 0, st, B);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(reduce_energy_kernel, dim3((ctx->K_pad + 255) / 256), dim3(256), 0, st, part,
                     nparts, ctx->K_pad, ctx->Ko, ctx->Ko_pad, ctx->Ku, ctx->nocc, ctx->nu, ctx->nb,
                     dL_dE);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // host tables are freed on return
  return e;
}

}  // namespace lrs
