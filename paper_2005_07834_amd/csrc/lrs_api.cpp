// C ABI of the screening library: argument validation (host, before any launch), device
// buffers, lazy operand layouts, quadrature terms, launch plans and timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "lrs_internal.h"

using namespace lrs;

namespace {

const double kHartreeEv = 27.211386245988;
const double kPi = 3.14159265358979323846;

lrs_status fail(lrs_ctx* ctx, lrs_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

#define HIP_OR_FAIL(ctx, expr)                                                        \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, LRS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

void release(lrs_ctx* ctx, DevBuf& b) {
  if (b.p) {
    (void)hipFree(b.p);
    ctx->bytes_in_use -= b.bytes;
  }
  b.p = nullptr;
  b.bytes = 0;
}

// Allocates (or keeps, if already large enough) a device buffer, honouring LRS_MAX_BYTES.
lrs_status ensure_buf(lrs_ctx* ctx, DevBuf& b, size_t bytes, const char* what) {
  bytes = (size_t)round_up((long long)std::max<size_t>(bytes, 256), 256);
  if (b.p && b.bytes >= bytes) return LRS_OK;
  if (ctx->capturing)
    return fail(ctx, LRS_ESTATE, "%s: the call would allocate during stream capture; run it "
                "once on the same problem before capturing", what);
  if (b.p && ctx->graph_pinned)
    return fail(ctx, LRS_ESTATE, "%s: the call would replace a buffer that captured graphs "
                "read; call lrs_release_graphs once those graphs are gone", what);
  release(ctx, b);
  if (ctx->max_bytes && ctx->bytes_in_use + bytes > ctx->max_bytes)
    return fail(ctx, LRS_ENOMEM, "%s: %zu bytes would exceed LRS_MAX_BYTES (%zu in use)", what,
                bytes, ctx->bytes_in_use);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(ctx, LRS_ENOMEM, "%s: hipMalloc of %zu bytes failed", what, bytes);
  }
  b.p = p;
  b.bytes = bytes;
  ctx->bytes_in_use += bytes;
  return LRS_OK;
}

#define CHECK(st)                 \
  do {                            \
    lrs_status s_ = (st);         \
    if (s_ != LRS_OK) return s_;  \
  } while (0)

bool all_finite(const double* x, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

void drop_plans(lrs_ctx* ctx) {
  for (auto& kv : ctx->plans) release(ctx, kv.second.tiles);
  ctx->plans.clear();
}

void drop_sites(lrs_ctx* ctx) {
  release(ctx, ctx->site_f64);
  release(ctx, ctx->a_tiles);
  ctx->a_prec = -1;
  release(ctx, ctx->psi_site_f64);
  release(ctx, ctx->psi_site_bf16);
  ctx->psi_kmajor_ok = ctx->psi_split_ok = false;
  for (auto& b : ctx->site_tiles) release(ctx, b);
  release(ctx, ctx->site_colmap);
  release(ctx, ctx->g_keep);
  ctx->g_keep_prec = -1;
  ctx->have_sites = false;
  ctx->have_W = false;
  ctx->have_rho = false;
  drop_plans(ctx);
}

void drop_quad(lrs_ctx* ctx) {
  release(ctx, ctx->w_nat);
  release(ctx, ctx->c_dev);
  ctx->a_prec = -1;
  ctx->g_keep_prec = -1;
  ctx->have_quad = false;
  ctx->quad = Quad();
}

// max |Im psi| over n complex values on the device (synchronises)
lrs_status device_max_abs_im(lrs_ctx* ctx, const double* psi, long long n, float* out) {
  DevBuf tmp;
  CHECK(ensure_buf(ctx, tmp, 256, "max|Im| scratch"));
  lrs_status st = LRS_OK;
  unsigned int h = 0;
  if (launch_fill_zero(tmp.p, 256, ctx->stream) != hipSuccess ||
      launch_max_abs_im(psi, n, (unsigned int*)tmp.p, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(&h, tmp.p, 4, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    st = fail(ctx, LRS_EDEVICE, "max|Im| reduction failed");
  release(ctx, tmp);
  std::memcpy(out, &h, 4);
  return st;
}

// max |x| over a device array of doubles, and whether any entry is not finite (synchronises)
lrs_status device_max_abs(lrs_ctx* ctx, const double* x, long long n, float* out, bool* bad) {
  DevBuf tmp;
  CHECK(ensure_buf(ctx, tmp, 256, "max|x| scratch"));
  lrs_status st = LRS_OK;
  unsigned int h[2] = {0, 0};
  if (launch_fill_zero(tmp.p, 256, ctx->stream) != hipSuccess ||
      launch_max_abs(x, n, (unsigned int*)tmp.p, ctx->stream) != hipSuccess ||
      hipMemcpyAsync(h, tmp.p, 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess)
    st = fail(ctx, LRS_EDEVICE, "max|x| reduction failed");
  release(ctx, tmp);
  float m;
  std::memcpy(&m, &h[0], 4);
  *out = m;
  *bad = h[1] != 0;
  return st;
}

float pow2_prescale(float maxabs) {
  if (!(maxabs > 0)) return 1.f;
  int e = (int)std::floor(std::log2((double)maxabs));
  return (float)std::ldexp(1.0, -e);
}

// ------------------------------------------------------------------ lazy operand layouts
lrs_status ensure_grid_tiles(lrs_ctx* ctx, int prec) {
  if (ctx->ngrid <= 0) return fail(ctx, LRS_ESTATE, "no grid orbitals were given");
  DevBuf& b = ctx->grid_tiles[prec];
  if (b.p) return LRS_OK;
  size_t bytes = (size_t)(ctx->grid_cols_pad / 16) * (ctx->K_pad / chunk_of(prec)) * tile_bytes(prec);
  CHECK(ensure_buf(ctx, b, bytes, "grid operand"));
  HIP_OR_FAIL(ctx, launch_repack_from_f64(ctx->grid_tiles[LRS_FP64].p, ctx->grid_cols_pad,
                                          ctx->K_pad, prec, ctx->grid_scale_f16, b.p,
                                          ctx->stream));
  return LRS_OK;
}

lrs_status ensure_site_tiles(lrs_ctx* ctx, int prec) {
  DevBuf& b = ctx->site_tiles[prec];
  if (b.p) return LRS_OK;
  size_t bytes = (size_t)(ctx->site_cols_pad / 16) * (ctx->K_pad / chunk_of(prec)) * tile_bytes(prec);
  CHECK(ensure_buf(ctx, b, bytes, "site column operand"));
  HIP_OR_FAIL(ctx, launch_site_col_tiles((const double*)ctx->site_f64.p, ctx->rows_pad,
                                         ctx->K_pad, ctx->site_cols_pad,
                                         (const int*)ctx->site_colmap.p, prec,
                                         ctx->site_scale_f16, b.p, ctx->stream));
  return LRS_OK;
}

// ------------------------------------------------------------------ quadrature terms
// alpha/beta given per term on the (k, band) grid; normalises each term's weights by powers
// of two (largest weight in [1, 2)) and moves the factors into c.
lrs_status install_terms(lrs_ctx* ctx, Quad& q, const std::vector<double>& c,
                         const std::vector<double>& alpha, const std::vector<double>& beta,
                         const std::vector<double>* dalpha, const std::vector<double>* dbeta,
                         const std::vector<double>* ci = nullptr) {
  const int T = (int)c.size();
  // real orbitals: weights per orbital (Kp = 2 K_pad of them, the unoccupied from 2 Ko_pad),
  // rearranged below into the slot layout
  const bool real = ctx->real_mode;
  const int Ko = ctx->Ko, Ku = ctx->Ku, Kp = real ? 2 * ctx->K_pad : ctx->K_pad;
  const int Ko_pad = real ? 2 * ctx->Ko_pad : ctx->Ko_pad;
  q.nterms = T;
  q.c_raw = c;
  q.c.assign(T, 0.0);
  q.ci.assign(ci ? T : 0, 0.0);
  q.w.assign((size_t)T * Kp, 0.0);
  q.dw.assign((size_t)T * Kp, 0.0);
  q.has_deriv = dalpha != nullptr;
  for (int t = 0; t < T; ++t) {
    double ma = 0, mb = 0;
    for (int i = 0; i < Ko; ++i) ma = std::max(ma, alpha[(size_t)t * Ko + i]);
    for (int i = 0; i < Ku; ++i) mb = std::max(mb, beta[(size_t)t * Ku + i]);
    // A term whose largest weight on either side is below 1e-200 contributes less than
    // c * 1e-200 to any band pair and is dropped (its power-of-two normalisation would
    // overflow); it stays in the list with zero weights.
    if (!(ma >= 1e-200) || !(mb >= 1e-200)) {
      q.c[t] = 0.0;
      continue;
    }
    double sa = std::ldexp(1.0, -(int)std::floor(std::log2(ma)));
    double sb = std::ldexp(1.0, -(int)std::floor(std::log2(mb)));
    q.c[t] = c[t] / (sa * sb);
    if (ci) q.ci[t] = (*ci)[t] / (sa * sb);
    double* w = &q.w[(size_t)t * Kp];
    double* dw = &q.dw[(size_t)t * Kp];
    for (int i = 0; i < Ko; ++i) {
      w[i] = alpha[(size_t)t * Ko + i] * sa;
      if (dalpha) dw[i] = (*dalpha)[(size_t)t * Ko + i] * sa;
    }
    for (int i = 0; i < Ku; ++i) {
      w[Ko_pad + i] = beta[(size_t)t * Ku + i] * sb;
      if (dbeta) dw[Ko_pad + i] = (*dbeta)[(size_t)t * Ku + i] * sb;
    }
  }
  if (real) {
    // slot k of chunk k / 16 holds orbitals 32 (k / 16) + k % 16 (re) and that + 16 (im): per
    // term the re orbitals' weights [K_pad], then the im orbitals' [K_pad]
    const int Ks = ctx->K_pad;
    std::vector<double> w2(q.w.size()), dw2(q.dw.size());
    for (int t = 0; t < T; ++t)
      for (int k = 0; k < Ks; ++k) {
        const int K = 32 * (k >> 4) + (k & 15);
        w2[(size_t)t * Kp + k] = q.w[(size_t)t * Kp + K];
        w2[(size_t)t * Kp + Ks + k] = q.w[(size_t)t * Kp + K + 16];
        dw2[(size_t)t * Kp + k] = q.dw[(size_t)t * Kp + K];
        dw2[(size_t)t * Kp + Ks + k] = q.dw[(size_t)t * Kp + K + 16];
      }
    q.w_orb.swap(q.w);
    q.dw_orb.swap(q.dw);
    q.w.swap(w2);
    q.dw.swap(dw2);
  }
  // device copies: weights in natural K order (real orbitals: the slot layout above; FP64) and
  // the coefficients
  CHECK(ensure_buf(ctx, ctx->w_nat, q.w.size() * 8, "weights"));
  CHECK(ensure_buf(ctx, ctx->c_dev, (size_t)2 * T * 8, "term coefficients"));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->w_nat.p, q.w.data(), q.w.size() * 8,
                                  hipMemcpyHostToDevice, ctx->stream));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->c_dev.p, q.c.data(), (size_t)T * 8,
                                  hipMemcpyHostToDevice, ctx->stream));
  if (ci)
    HIP_OR_FAIL(ctx, hipMemcpyAsync((double*)ctx->c_dev.p + T, q.ci.data(), (size_t)T * 8,
                                    hipMemcpyHostToDevice, ctx->stream));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));   // host vectors are freed on return
  ctx->have_quad = true;
  ++ctx->quad_version;
  drop_plans(ctx);
  return LRS_OK;
}

// x = mu - e_occ > 0, y = e_unocc - mu > 0 (lrs_check_bands put every band on its label's
// side of mu), with the metallic regularisation of Sec. VI.D: mu - e keeps its sign and takes
// delta in quadrature, so x -> sqrt(x^2 + delta^2) and y -> sqrt(y^2 + delta^2)
void offsets(const lrs_ctx* ctx, std::vector<double>& x, std::vector<double>& y) {
  x.resize(ctx->Ko);
  y.resize(ctx->Ku);
  const double d2 = ctx->delta > 0 ? ctx->delta * ctx->delta : 0.0;
  for (int k = 0; k < ctx->nk; ++k) {
    for (int n = 0; n < ctx->nocc; ++n) {
      const double v = ctx->mu - ctx->energies[(size_t)k * ctx->nb + n];
      x[(size_t)k * ctx->nocc + n] = d2 > 0 ? std::sqrt(v * v + d2) : v;
    }
    for (int m = 0; m < ctx->nu; ++m) {
      const double v = ctx->energies[(size_t)k * ctx->nb + ctx->nocc + m] - ctx->mu;
      y[(size_t)k * ctx->nu + m] = d2 > 0 ? std::sqrt(v * v + d2) : v;
    }
  }
}

// ------------------------------------------------------------------ plans
long long plan_key(int site, int cols, int prec, int variant, int mode) {
  return ((((long long)(site + 1) * 4 + cols) * 8 + prec) * 16 + variant) * 2 + mode;
}

// Bytes of weighted site operand per 16-row block for nt terms.
size_t a_bytes_per_rb(const lrs_ctx* ctx, int prec, int nt) {
  return (size_t)nt * (ctx->K_pad / chunk_of(prec)) * tile_bytes(prec);
}

size_t a_budget() {
  if (const char* e = std::getenv("LRS_SITE_OPERAND_BYTES")) return (size_t)std::strtoull(e, nullptr, 10);
  return (size_t)24 << 30;
}

lrs_status get_plan(lrs_ctx* ctx, int site, int cols, int prec, int variant, int mode,
                    Plan** out) {
  long long key = plan_key(site, cols, prec, variant, mode);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) {
    *out = &it->second;
    return LRS_OK;
  }
  if (ctx->capturing)
    return fail(ctx, LRS_ESTATE, "the tile plan would be built during stream capture; run the "
                "call once on the same problem before capturing");
  TileShape sh = chi0_shape(prec, variant);
  if (kRowAlign % sh.bm != 0) return fail(ctx, LRS_EINVAL, "tile rows must divide %d", kRowAlign);
  const int nt = mode == 1 ? 1 : ctx->quad.nterms;
  const size_t per_rb = a_bytes_per_rb(ctx, prec, nt);
  int max_rb = (int)std::min<size_t>(1 << 20, a_budget() / std::max<size_t>(per_rb, 1));
  max_rb = std::max(kRowAlign / 16, max_rb / (kRowAlign / 16) * (kRowAlign / 16));
  const int s0 = site < 0 ? 0 : site, s1 = site < 0 ? ctx->nsites : site + 1;
  // 1. the sites' rows in tiles of bm rows (128-row slots hold 128/bm of them), cut into
  //    batches at max_rb row blocks of weighted site operand
  struct RowTile {
    int site, slot_row, rows, m0;   // m0: first row within the site
  };
  std::vector<std::vector<RowTile>> brows(1);
  Plan p;
  p.variant = variant;
  Batch cur;
  cur.rb0 = ctx->site_col_off[s0] / 16;
  for (int s = s0; s < s1; ++s) {
    const int n = ctx->site_off[s + 1] - ctx->site_off[s];
    const int slot0 = ctx->site_col_off[s];
    for (int m0 = 0; m0 < n; m0 += kRowAlign) {
      const int rb = (slot0 + m0) / 16;
      if (rb + kRowAlign / 16 - cur.rb0 > max_rb && rb > cur.rb0) {
        cur.nrb = rb - cur.rb0;
        p.batches.push_back(cur);
        brows.emplace_back();
        cur = Batch();
        cur.rb0 = rb;
      }
      for (int r = m0; r < std::min(n, m0 + kRowAlign); r += sh.bm)
        brows.back().push_back(RowTile{s, slot0 + r, std::min(sh.bm, n - r), r});
    }
  }
  const int last_slot = ctx->site_col_off[s1 - 1] +
                        (int)round_up(ctx->site_off[s1] - ctx->site_off[s1 - 1], kRowAlign);
  cur.nrb = last_slot / 16 - cur.rb0;
  p.batches.push_back(cur);
  // 2. tiles in 2-D blocks: the workgroups of one XCD run 32 consecutive tiles of the list
  //    at a time and the whole grid runs 256, so the list goes in 16 x 16 blocks of
  //    (row tile, column tile), each made of eight BR x BC blocks (BR BC = 32): the
  //    concurrent tiles of an XCD then share BR A and BC B panels in its L2, and those of
  //    the grid 16 + 16 in the memory-side cache, instead of one row against hundreds of
  //    columns.  A panel chunk is bm rows and a B one bn columns, so BR is the power of two
  //    that minimises the bytes BR bm + BC bn an XCD fetches per chunk step (4 x 8 for square
  //    tiles, 8 x 4 for 128 x 192).
  std::vector<TileDesc> tiles;
  int BR = 4;
  for (int br = 1; br <= 32; br *= 2)
    if ((long long)br * sh.bm + (32 / br) * sh.bn < (long long)BR * sh.bm + (32 / BR) * sh.bn)
      BR = br;
  const int BC = 32 / BR;
  auto emit_blocked = [&](int nr, int nc, auto&& make) {
    constexpr int SR = 16, SC = 16;
    for (int R0 = 0; R0 < nr; R0 += SR)
      for (int C0 = 0; C0 < nc; C0 += SC) {
        const int R1 = std::min(nr, R0 + SR), C1 = std::min(nc, C0 + SC);
        for (int r1 = R0; r1 < R1; r1 += BR)
          for (int c1 = C0; c1 < C1; c1 += BC)
            for (int r = r1; r < std::min(R1, r1 + BR); ++r)
              for (int c = c1; c < std::min(C1, c1 + BC); ++c) make(r, c);
      }
  };
  // site-block output offsets; the adjoint mode (1) writes blocks with rows padded to a
  // multiple of kAdjAlign (site_block_ld), the layout its GEMMs read
  std::vector<long long> site_base(ctx->nsites + 1, 0);
  for (int s = s0; s < s1; ++s) {
    const long long ld = site_block_ld(ctx->site_off[s + 1] - ctx->site_off[s], mode);
    site_base[s + 1] = site_base[s] + ld * ld;
  }
  for (size_t bi = 0; bi < p.batches.size(); ++bi) {
    Batch& bt = p.batches[bi];
    const std::vector<RowTile>& rt = brows[bi];
    bt.tile0 = (int)tiles.size();
    if (cols == LRS_COLS_GRID) {
      const int ng = ctx->ngrid, nc = (ng + sh.bn - 1) / sh.bn;
      emit_blocked((int)rt.size(), nc, [&](int r, int c) {
        const RowTile& x = rt[r];
        const long long orow = ctx->site_off[x.site] - ctx->site_off[s0] + x.m0;
        TileDesc t;
        t.a_row0 = x.slot_row - bt.rb0 * 16;
        t.b_col0 = c * sh.bn;
        t.nrows = x.rows;
        t.ncols = std::min(sh.bn, ng - c * sh.bn);
        t.out_off = orow * ng + (long long)c * sh.bn;
        t.ldo = ng;
        t.pad = 0;
        t.m0 = t.c0 = 0;
        tiles.push_back(t);
      });
    } else {
      // each site's square block on its own (its columns are its own points)
      for (size_t i = 0; i < rt.size();) {
        size_t j = i;
        while (j < rt.size() && rt[j].site == rt[i].site) ++j;
        const int s = rt[i].site;
        const int n = ctx->site_off[s + 1] - ctx->site_off[s];
        const int slot0 = ctx->site_col_off[s];
        const int nc = (n + sh.bn - 1) / sh.bn;
        const int ld = site_block_ld(n, mode);
        emit_blocked((int)(j - i), nc, [&](int r, int c) {
          const RowTile& x = rt[i + r];
          // chi0 (symmetric) and the adjoint's H (Hermitian) blocks are stored from their
          // upper triangle: tiles wholly below the diagonal are not needed, and pad carries
          // (first row - first column).  Mode 2 (chi0 at imaginary frequency, whose odd part
          // is antisymmetric) lists every tile.
          if (mode != 2 && c * sh.bn + sh.bn - 1 < x.m0) return;
          TileDesc t;
          t.a_row0 = x.slot_row - bt.rb0 * 16;
          t.b_col0 = slot0 + c * sh.bn;
          t.nrows = x.rows;
          t.ncols = std::min(sh.bn, n - c * sh.bn);
          t.out_off = site_base[s] - site_base[s0] + (long long)x.m0 * ld + (long long)c * sh.bn;
          t.ldo = ld;
          t.pad = x.m0 - c * sh.bn;
          t.m0 = x.m0;
          t.c0 = c * sh.bn;
          tiles.push_back(t);
        });
        i = j;
      }
    }
    bt.ntiles = (int)tiles.size() - bt.tile0;
  }
  p.ntiles = (int)tiles.size();
  // every tile's operand reads (bm rows of its batch's A, bn columns of B) stay inside the
  // operands; the kernel does not check them
  {
    const int b_cols = cols == LRS_COLS_GRID ? ctx->grid_cols_pad : ctx->site_cols_pad;
    for (const Batch& b : p.batches)
      for (int i = b.tile0; i < b.tile0 + b.ntiles; ++i) {
        const TileDesc& t = tiles[i];
        if (t.a_row0 < 0 || t.a_row0 % 16 || t.a_row0 + sh.bm > b.nrb * 16 || t.b_col0 < 0 ||
            t.b_col0 % 16 || t.b_col0 + sh.bn > b_cols || t.nrows <= 0 || t.ncols <= 0)
          return fail(ctx, LRS_EINVAL, "internal: tile %d exceeds its operands", i);
      }
  }
  int per_cu = chi0_blocks_per_cu(prec, variant);
  long long maxg = (long long)ctx->num_cu * std::max(1, per_cu);
  for (auto& b : p.batches) {
    long long g = std::min<long long>(maxg, round_up(std::max(b.ntiles, 1), 8));
    b.grid = (int)std::max<long long>(8, g / 8 * 8);
  }
  p.area.assign(tiles.size() + 1, 0);
  for (size_t i = 0; i < tiles.size(); ++i)
    p.area[i + 1] = p.area[i] + (long long)tiles[i].nrows * tiles[i].ncols;
  CHECK(ensure_buf(ctx, p.tiles, tiles.size() * sizeof(TileDesc) + 32, "tile list"));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(p.tiles.p, tiles.data(), tiles.size() * sizeof(TileDesc),
                                  hipMemcpyHostToDevice, ctx->stream));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
  auto res = ctx->plans.emplace(key, p);
  *out = &res.first->second;
  return LRS_OK;
}

// Weighted site operand of terms [t0, t0+nt) for one batch (kept while nothing changes).
// The weighted site operand of terms [t0, t0 + nt) for the rows of batch b; *a is the first
// term's part.  The context keeps one operand: a request that the kept one covers (same
// precision, terms, batch rows; terms are stored one after the other) uses it in place, so the
// adjoint's one-term requests reuse the all-term operand of the forward launches.
lrs_status site_operand(lrs_ctx* ctx, int prec, const Batch& b, int t0, int nt,
                        const void** a = nullptr) {
  // Under capture the graph must build the operand itself (a replay cannot rely on what the
  // buffer held at capture time); while graphs are pinned their replays rewrite the buffer in
  // stream order, so the kept operand is never trusted then either.
  if (ctx->capturing || ctx->graph_pinned) ctx->a_prec = -1;
  if (ctx->a_prec == prec && ctx->a_version == ctx->quad_version && ctx->a_rb0 == b.rb0 &&
      ctx->a_nrb == b.nrb && ctx->a_t0 <= t0 && t0 + nt <= ctx->a_t0 + ctx->a_nt &&
      ctx->a_tiles.p) {
    if (a)
      *a = (const unsigned char*)ctx->a_tiles.p +
           (size_t)(t0 - ctx->a_t0) * a_bytes_per_rb(ctx, prec, 1) * b.nrb;
    return LRS_OK;
  }
  ctx->a_prec = -1;
  CHECK(ensure_buf(ctx, ctx->a_tiles, a_bytes_per_rb(ctx, prec, nt) * b.nrb, "weighted site operand"));
  const double a_scale = is_f16(prec) ? ctx->site_scale_f16 : 1.0;
  // (real orbitals: the weights of a slot's second orbital follow those of the first)
  const int w_stride = ctx->real_mode ? 2 * ctx->K_pad : ctx->K_pad;
  const int q_woff = ctx->real_mode ? ctx->K_pad : 0;
  HIP_OR_FAIL(ctx, launch_prep_site(prec, (const double*)ctx->site_f64.p, ctx->rows_pad,
                                    ctx->K_pad, (const int*)ctx->site_colmap.p, b.rb0, b.nrb,
                                    (const double*)ctx->w_nat.p, w_stride, q_woff, t0, nt,
                                    a_scale, ctx->a_tiles.p, ctx->stream));
  ctx->a_prec = prec;
  ctx->a_version = ctx->quad_version;
  ctx->a_rb0 = b.rb0;
  ctx->a_nrb = b.nrb;
  ctx->a_t0 = t0;
  ctx->a_nt = nt;
  if (a) *a = ctx->a_tiles.p;
  return LRS_OK;
}

lrs_status park_for(lrs_ctx* ctx, int prec, int variant, int grid) {
  const size_t bytes = chi0_shape(prec, variant).park_bytes * (size_t)grid;
  return ensure_buf(ctx, ctx->park, bytes, "G_o scratch");
}

int pick_variant(lrs_ctx* ctx, int prec, int cols) {
  const char* e = std::getenv("LRS_VARIANT");
  if (e) {
    int v = std::atoi(e);
    if (v >= 0 && v < chi0_num_variants(prec)) return v;
  }
  if (ctx->tuned_variant[prec][cols] >= 0) return ctx->tuned_variant[prec][cols];
  return chi0_default_variant(prec);
}

// max_tiles > 0 limits the launch to the first tiles of the first batch (tuning samples)
lrs_status run_chi0(lrs_ctx* ctx, int site, int cols, int prec, int variant, double* out,
                    bool timed, int max_tiles = 0) {
  Plan* plan = nullptr;
  const bool odd = !ctx->quad.ci.empty();    // complex term coefficients (imaginary frequency)
  CHECK(get_plan(ctx, site, cols, prec, variant, cols == LRS_COLS_SITE && odd ? 2 : 0, &plan));
  double bscale = 1.0;
  const void* b;
  const int b_ncb = (cols == LRS_COLS_GRID ? ctx->grid_cols_pad : ctx->site_cols_pad) / 16;
  if (cols == LRS_COLS_GRID) {
    CHECK(ensure_grid_tiles(ctx, prec));
    b = ctx->grid_tiles[prec].p;
    if (is_f16(prec)) bscale = ctx->grid_scale_f16;
  } else {
    CHECK(ensure_site_tiles(ctx, prec));
    b = ctx->site_tiles[prec].p;
    if (is_f16(prec)) bscale = ctx->site_scale_f16;
  }
  const double a_scale = is_f16(prec) ? ctx->site_scale_f16 : 1.0;
  const int KC = chunk_of(prec);
  const int nch = ctx->K_pad / KC;
  double pref = -2.0 * ctx->spin / ((double)ctx->nk * ctx->nk);
  const double g_scale = a_scale * bscale;   // each G carries a_scale * b_scale
  pref /= g_scale * g_scale;
  const int T = ctx->quad.nterms;
  // an F16F8, BF16X2 or FP64 launch over every site block keeps each term's Green's functions
  // for the adjoint (which would otherwise recompute them) when they fit in kKeepMaxBytes; the
  // adjoint's own launch would form them in the same order (not so a rotating-B variant's)
  void* keep_o = nullptr;
  void* keep_u = nullptr;
  long long keep_stride = 0;
  const bool keeps = prec == LRS_F16F8 || prec == LRS_FP64 ||
                     (prec == LRS_BF16X2 && !chi0_variant_rotates(prec, variant));
  const size_t keep_elem = prec == LRS_FP64 ? 16 : 8;
  if (cols == LRS_COLS_SITE && site < 0 && keeps && max_tiles == 0 && !ctx->capturing) {
    for (int s = 0; s < ctx->nsites; ++s) {
      const long long n = ctx->site_off[s + 1] - ctx->site_off[s];
      keep_stride += n * n;
    }
    const size_t bytes = (size_t)2 * T * keep_stride * keep_elem;
    ctx->g_keep_prec = -1;
    if (bytes <= kKeepMaxBytes && ensure_buf(ctx, ctx->g_keep, bytes, "kept G") == LRS_OK) {
      keep_o = ctx->g_keep.p;
      keep_u = (char*)ctx->g_keep.p + (size_t)T * keep_stride * keep_elem;
    } else {
      ctx->err.clear();     // (not kept: the adjoint recomputes them)
    }
  }
  bool first = true;
  for (const Batch& bt : plan->batches) {
    if (bt.ntiles == 0) continue;
    const void* a_op = nullptr;
    CHECK(site_operand(ctx, prec, bt, 0, T, &a_op));
    int nt = bt.ntiles, grid = bt.grid;
    if (max_tiles > 0) {
      nt = std::min(nt, max_tiles);
      grid = (int)std::max<long long>(8, std::min<long long>(grid, round_up(nt, 8)));
    }
    CHECK(park_for(ctx, prec, variant, grid));
    // the workgroups of each XCD meet at every term start (LRS_XCD_SYNC=0 turns this off);
    // the counters start from zero in every launch
    unsigned int* sync = nullptr;
    const char* se = std::getenv("LRS_XCD_SYNC");
    if (!se || std::atoi(se) != 0) {
      CHECK(ensure_buf(ctx, ctx->xcd_sync, 8 * 64, "XCD counters"));
      sync = (unsigned int*)ctx->xcd_sync.p;
      HIP_OR_FAIL(ctx, launch_fill_zero(sync, 8 * 64, ctx->stream));
    }
    if (timed && first) HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    first = false;
    HIP_OR_FAIL(ctx, launch_chi0(prec, variant, grid, a_op, bt.nrb, b, b_ncb, nch,
                                 (const double*)ctx->c_dev.p,
                                 odd ? (const double*)ctx->c_dev.p + T : nullptr, T,
                                 ctx->Ko_pad / KC, (const TileDesc*)plan->tiles.p + bt.tile0, nt,
                                 out, pref, cols == LRS_COLS_SITE && !odd, sync, ctx->park.p,
                                 ctx->real_mode ? 1 : 0, keep_o, keep_u, keep_stride,
                                 ctx->stream));
    if (max_tiles > 0) break;
  }
  if (timed && !first) {
    HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    ctx->timed = true;
  }
  if (keep_o) ctx->g_keep_prec = prec;
  return LRS_OK;
}

}  // namespace

namespace lrs {
lrs_status plan_for(lrs_ctx* ctx, int site, int cols, int prec, int variant, int mode,
                    Plan** out) {
  return get_plan(ctx, site, cols, prec, variant, mode, out);
}
lrs_status ensure_site_tiles_for(lrs_ctx* ctx, int prec) { return ensure_site_tiles(ctx, prec); }
lrs_status ensure_site_operand(lrs_ctx* ctx, int prec, const Batch& b, int t0, int nt,
                               const void** a) {
  return site_operand(ctx, prec, b, t0, nt, a);
}
lrs_status ensure_park(lrs_ctx* ctx, int prec, int variant, int grid) {
  return park_for(ctx, prec, variant, grid);
}
}  // namespace lrs

// ====================================================================== C ABI
extern "C" {

const char* lrs_version(void) { return "lrs 0.1 (gfx950)"; }

lrs_status lrs_create(lrs_ctx** out, int device, void* hip_stream) {
  if (!out) return LRS_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return LRS_EDEVICE;
  }
  if (device < 0 || device >= n) return LRS_EINVAL;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return LRS_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LRS_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return LRS_EDEVICE;
  // the allocation-free solve's fixed scratch array: its address on this device, once
  if (scratch_setup(device) != hipSuccess) {
    (void)hipGetLastError();
    return LRS_EDEVICE;
  }
  lrs_ctx* ctx = new lrs_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->num_cu = prop.multiProcessorCount;
  if (const char* e = std::getenv("LRS_MAX_BYTES")) ctx->max_bytes = (size_t)std::strtoull(e, nullptr, 10);
  if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess) {
    delete ctx;
    return LRS_EDEVICE;
  }
  *out = ctx;
  return LRS_OK;
}

void lrs_destroy(lrs_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  drop_sites(ctx);
  drop_quad(ctx);
  for (auto& b : ctx->grid_tiles) release(ctx, b);
  release(ctx, ctx->W_last);
  release(ctx, ctx->rho_last);
  release(ctx, ctx->screen_tab);
  release(ctx, ctx->work);
  release(ctx, ctx->adj_work);
  release(ctx, ctx->val_work);
  release(ctx, ctx->fft_work);
  release(ctx, ctx->probe);
  release(ctx, ctx->proj_work);
  release(ctx, ctx->a_tiles);
  release(ctx, ctx->park);
  release(ctx, ctx->g_keep);
  release(ctx, ctx->xcd_sync);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  delete ctx;
}

const char* lrs_last_error(const lrs_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

lrs_status lrs_check_bands(int nk, int nb, int nocc, const double* e, double mu, double delta) {
  if (nk < 1 || nb < 2 || nocc < 1 || nocc >= nb || !e) return LRS_EINVAL;
  if (!(delta >= 0) || !std::isfinite(delta)) return LRS_EINVAL;
  if (!all_finite(e, (size_t)nk * nb)) return LRS_ENONFINITE;
  if (std::isinf(mu)) return LRS_ENONFINITE;
  double top = -INFINITY, bottom = INFINITY;
  for (int k = 0; k < nk; ++k) {
    for (int n = 0; n < nocc; ++n) top = std::max(top, e[(size_t)k * nb + n]);
    for (int m = nocc; m < nb; ++m) bottom = std::min(bottom, e[(size_t)k * nb + m]);
  }
  // The side of mu decides occupation (Sec. VI.D; the metallic regularisation keeps the sign
  // of mu - e).  The lowest nocc bands are occupied at every k, so every one of them must lie
  // below mu and every other band above it.  Without regularisation a band set that allows no
  // such mu has no gap; with it, such a set (a metal whose occupied count changes with k) is
  // a case this library does not implement.
  const lrs_status side = delta > 0 ? LRS_EUNSUPPORTED : LRS_ENOGAP;
  if (!(bottom > top)) return side;
  if (!std::isnan(mu) && !(mu > top && mu < bottom)) return side;
  return LRS_OK;
}

namespace {
// lrs_set_orbitals, and with real != 0 lrs_set_orbitals_real
lrs_status set_orbitals_impl(lrs_ctx* ctx, int nk, int nb, int nocc, int spin_factor,
                             const double* e, double mu, double delta, const void* psi_grid,
                             int ngrid, double grid_dV, int real) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (ctx->graph_pinned)
    return fail(ctx, LRS_ESTATE, "captured graphs read this context's buffers; call "
                "lrs_release_graphs once those graphs are gone");
  lrs_status st = lrs_check_bands(nk, nb, nocc, e, mu, delta);
  if (st == LRS_EINVAL) return fail(ctx, st, "invalid band set (nk=%d nb=%d nocc=%d delta=%g)", nk, nb, nocc, delta);
  if (st == LRS_ENONFINITE) return fail(ctx, st, "non-finite band energy or mu");
  if (st == LRS_ENOGAP) return fail(ctx, st, "no global gap between occupied and unoccupied bands (or mu outside it)");
  if (st == LRS_EUNSUPPORTED)
    return fail(ctx, st, "with delta > 0 a band labelled occupied lies above mu or an unoccupied "
                "one below it: occupied counts that change with k are not supported");
  if (spin_factor != 1 && spin_factor != 2) return fail(ctx, LRS_EINVAL, "spin_factor must be 1 or 2");
  if (ngrid < 0 || (ngrid > 0 && !psi_grid) || (ngrid == 0 && psi_grid))
    return fail(ctx, LRS_EINVAL, "psi_grid and ngrid must be given together");
  if (ngrid > 0 && !(grid_dV > 0)) return fail(ctx, LRS_EINVAL, "grid_dV must be > 0");
  const long long K = (long long)nk * nb;
  if (K > (1LL << 26) || (long long)ngrid > (1LL << 28)) return fail(ctx, LRS_EINVAL, "problem too large");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));

  // sizes and storage for the new state, validated before the old state is dropped
  const int Ko = nk * nocc, Ku = nk * (nb - nocc);
  // (real orbitals: two per slot, so the orbital counts are padded to twice the alignment)
  const int align = real ? 2 * kPhaseAlign : kPhaseAlign;
  const int Ko_pad = (int)round_up(Ko, align) / (real ? 2 : 1);
  const int Ku_pad = (int)round_up(Ku, align) / (real ? 2 : 1);
  const int K_pad = Ko_pad + Ku_pad;
  const int cols_pad = ngrid > 0 ? (int)round_up(ngrid, kRowAlign) + kMaxTileCols : 0;
  DevBuf tiles;
  if (ngrid > 0) {
    size_t bytes = (size_t)(cols_pad / 16) * (K_pad / kChunkF64) * kTileBytes;
    CHECK(ensure_buf(ctx, tiles, bytes, "grid operand fp64"));
    float m = 0;
    bool bad = false;
    lrs_status s2 = device_max_abs(ctx, (const double*)psi_grid, 2LL * K * ngrid, &m, &bad);
    if (s2 != LRS_OK || bad) {
      release(ctx, tiles);
      return s2 != LRS_OK ? s2 : fail(ctx, LRS_ENONFINITE, "non-finite value in psi_grid");
    }
    if (real) {
      float mi = 0;
      lrs_status s3 = device_max_abs_im(ctx, (const double*)psi_grid, K * ngrid, &mi);
      if (s3 != LRS_OK || !(mi <= 1e-12f * m)) {
        release(ctx, tiles);
        return s3 != LRS_OK ? s3 : fail(ctx, LRS_EINVAL, "psi_grid is not real: max|Im| %g "
                                        "against max|Re| %g", mi, m);
      }
    }
    ctx->grid_max_abs = m;
    hipError_t he = launch_pack_tiles((const double*)psi_grid, nk, nb, nocc, ngrid, ngrid, cols_pad,
                                      Ko_pad, K_pad, LRS_FP64, 1.f, real, tiles.p, ctx->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
    if (he != hipSuccess) {
      release(ctx, tiles);
      return fail(ctx, LRS_EDEVICE, "packing grid orbitals: %s", hipGetErrorString(he));
    }
  }
  drop_sites(ctx);
  drop_quad(ctx);
  for (auto& b : ctx->grid_tiles) release(ctx, b);
  ctx->grid_tiles[LRS_FP64] = tiles;
  ctx->nk = nk;
  ctx->nb = nb;
  ctx->nocc = nocc;
  ctx->nu = nb - nocc;
  ctx->spin = spin_factor;
  ctx->delta = delta;
  ctx->energies.assign(e, e + (size_t)nk * nb);
  double top = -INFINITY, bottom = INFINITY;
  for (int k = 0; k < nk; ++k) {
    for (int n = 0; n < nocc; ++n) top = std::max(top, e[(size_t)k * nb + n]);
    for (int m = nocc; m < nb; ++m) bottom = std::min(bottom, e[(size_t)k * nb + m]);
  }
  ctx->mu = std::isnan(mu) ? 0.5 * (top + bottom) : mu;
  ctx->Ko = Ko;
  ctx->Ku = Ku;
  ctx->Ko_pad = Ko_pad;
  ctx->Ku_pad = Ku_pad;
  ctx->K_pad = K_pad;
  ctx->ngrid = ngrid;
  ctx->grid_dV = grid_dV;
  ctx->grid_cols_pad = cols_pad;
  ctx->grid_scale_f16 = pow2_prescale(ctx->grid_max_abs);
  ctx->real_mode = real != 0;
  ctx->have_bands = true;
  return LRS_OK;
}
}  // namespace

lrs_status lrs_set_orbitals(lrs_ctx* ctx, int nk, int nb, int nocc, int spin_factor,
                            const double* e, double mu, double delta, const void* psi_grid,
                            int ngrid, double grid_dV) {
  return set_orbitals_impl(ctx, nk, nb, nocc, spin_factor, e, mu, delta, psi_grid, ngrid,
                           grid_dV, 0);
}

lrs_status lrs_set_orbitals_real(lrs_ctx* ctx, int nk, int nb, int nocc, int spin_factor,
                                 const double* e, double mu, double delta, const void* psi_grid,
                                 int ngrid, double grid_dV) {
  return set_orbitals_impl(ctx, nk, nb, nocc, spin_factor, e, mu, delta, psi_grid, ngrid,
                           grid_dV, 1);
}

lrs_status lrs_set_sites(lrs_ctx* ctx, int nsites, const int* nrad, const int* nang,
                         const double* radii, const double* rad_w, const double* ang_xyz,
                         const double* ang_w, const void* psi_site, int lmax) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (ctx->graph_pinned)
    return fail(ctx, LRS_ESTATE, "captured graphs read this context's buffers; call "
                "lrs_release_graphs once those graphs are gone");
  if (!ctx->have_bands) return fail(ctx, LRS_ESTATE, "lrs_set_orbitals must come first");
  if (nsites < 1 || !nrad || !nang || !radii || !rad_w || !ang_xyz || !ang_w || !psi_site)
    return fail(ctx, LRS_EINVAL, "missing site arguments");
  if (lmax < 0 || lmax > 2) return fail(ctx, LRS_EINVAL, "lmax must be 0..2");
  long long nrows = 0, trad = 0, tang = 0;
  for (int s = 0; s < nsites; ++s) {
    if (nrad[s] < 1 || nang[s] < 1 || nrad[s] > 4096 || nang[s] > 4096)
      return fail(ctx, LRS_EINVAL, "site %d: bad grid %d x %d", s, nrad[s], nang[s]);
    nrows += (long long)nrad[s] * nang[s];
    trad += nrad[s];
    tang += nang[s];
  }
  if (nrows > (1LL << 24)) return fail(ctx, LRS_EINVAL, "too many site points");
  if (!all_finite(radii, trad) || !all_finite(rad_w, trad) || !all_finite(ang_xyz, 3 * tang) ||
      !all_finite(ang_w, tang))
    return fail(ctx, LRS_ENONFINITE, "non-finite site geometry");
  for (long long i = 0; i < trad; ++i)
    if (!(radii[i] > 0)) return fail(ctx, LRS_EINVAL, "radii must be > 0");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  float m = 0;
  bool bad = false;
  CHECK(device_max_abs(ctx, (const double*)psi_site, 2LL * ctx->nk * ctx->nb * nrows, &m, &bad));
  if (bad) return fail(ctx, LRS_ENONFINITE, "non-finite value in psi_site");
  if (ctx->real_mode) {
    float mi = 0;
    CHECK(device_max_abs_im(ctx, (const double*)psi_site, (long long)ctx->nk * ctx->nb * nrows,
                            &mi));
    if (!(mi <= 1e-12f * m))
      return fail(ctx, LRS_EINVAL, "psi_site is not real (the orbitals were set real): max|Im| "
                  "%g against max|Re| %g", mi, m);
  }

  drop_sites(ctx);
  ctx->nsites = nsites;
  ctx->lmax = lmax;
  ctx->nrad.assign(nrad, nrad + nsites);
  ctx->nang.assign(nang, nang + nsites);
  ctx->radii.assign(radii, radii + trad);
  ctx->rad_w.assign(rad_w, rad_w + trad);
  ctx->ang_xyz.assign(ang_xyz, ang_xyz + 3 * tang);
  ctx->ang_w.assign(ang_w, ang_w + tang);
  ctx->site_off.assign(nsites + 1, 0);
  ctx->site_col_off.assign(nsites + 1, 0);
  ctx->rad_off.assign(nsites + 1, 0);
  ctx->ang_off.assign(nsites + 1, 0);
  for (int s = 0; s < nsites; ++s) {
    int n = nrad[s] * nang[s];
    ctx->site_off[s + 1] = ctx->site_off[s] + n;
    ctx->site_col_off[s + 1] = ctx->site_col_off[s] + (int)round_up(n, kRowAlign);
    ctx->rad_off[s + 1] = ctx->rad_off[s] + nrad[s];
    ctx->ang_off[s + 1] = ctx->ang_off[s] + nang[s];
  }
  ctx->nrows = (int)nrows;
  ctx->rows_pad = (int)round_up(nrows, kRowAlign) + kRowAlign;
  ctx->site_cols_pad = ctx->site_col_off[nsites] + kMaxTileCols;
  ctx->site_max_abs = m;
  ctx->site_scale_f16 = pow2_prescale(m);
  // column map of the site column operand: padded column -> site row (-1 = zero column)
  std::vector<int> colmap(ctx->site_cols_pad, -1);
  for (int s = 0; s < nsites; ++s)
    for (int i = 0; i < ctx->site_off[s + 1] - ctx->site_off[s]; ++i)
      colmap[ctx->site_col_off[s] + i] = ctx->site_off[s] + i;
  CHECK(ensure_buf(ctx, ctx->site_colmap, colmap.size() * sizeof(int), "site column map"));
  CHECK(ensure_buf(ctx, ctx->site_f64, (size_t)2 * ctx->rows_pad * ctx->K_pad * 8, "site operand"));
  HIP_OR_FAIL(ctx, hipMemcpyAsync(ctx->site_colmap.p, colmap.data(), colmap.size() * sizeof(int),
                                  hipMemcpyHostToDevice, ctx->stream));
  HIP_OR_FAIL(ctx, launch_pack_site_rows((const double*)psi_site, ctx->nk, ctx->nb, ctx->nocc,
                                         ctx->nrows, ctx->rows_pad, ctx->Ko_pad, ctx->K_pad,
                                         ctx->real_mode ? 1 : 0, (double*)ctx->site_f64.p,
                                         ctx->stream));
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream));
  ctx->have_sites = true;
  return LRS_OK;
}

lrs_status lrs_set_quadrature(lrs_ctx* ctx, int nterms, const double* c, const double* alpha,
                              const double* beta) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (ctx->graph_pinned)
    return fail(ctx, LRS_ESTATE, "captured graphs read this context's buffers; call "
                "lrs_release_graphs once those graphs are gone");
  if (!ctx->have_bands) return fail(ctx, LRS_ESTATE, "lrs_set_orbitals must come first");
  if (nterms < 1 || nterms > kMaxTerms || !c || !alpha || !beta)
    return fail(ctx, LRS_EINVAL, "nterms must be 1..%d with all arrays given", kMaxTerms);
  const size_t na = (size_t)nterms * ctx->Ko, nb_ = (size_t)nterms * ctx->Ku;
  if (!all_finite(c, nterms) || !all_finite(alpha, na) || !all_finite(beta, nb_))
    return fail(ctx, LRS_ENONFINITE, "non-finite quadrature term");
  for (int t = 0; t < nterms; ++t)
    if (!(c[t] > 0)) return fail(ctx, LRS_EINVAL, "c must be > 0");
  for (size_t i = 0; i < na; ++i)
    if (alpha[i] < 0) return fail(ctx, LRS_EINVAL, "alpha must be >= 0");
  for (size_t i = 0; i < nb_; ++i)
    if (beta[i] < 0) return fail(ctx, LRS_EINVAL, "beta must be >= 0");
  Quad q;
  q.kind = -1;
  q.scale = 0;
  q.tau.assign(nterms, 0.0);
  std::vector<double> cv(c, c + nterms), av(alpha, alpha + na), bv(beta, beta + nb_);
  drop_quad(ctx);
  CHECK(install_terms(ctx, q, cv, av, bv, nullptr, nullptr));
  ctx->quad = q;
  return LRS_OK;
}

static lrs_status make_quadrature(lrs_ctx* ctx, int kind, int nnodes, double scale,
                                  double omega);

lrs_status lrs_make_quadrature(lrs_ctx* ctx, int kind, int nnodes, double scale) {
  return make_quadrature(ctx, kind, nnodes, scale, 0.0);
}

lrs_status lrs_make_quadrature_iw(lrs_ctx* ctx, int nnodes, double scale, double omega) {
  if (ctx && !(std::isfinite(omega) && omega >= 0)) {
    ctx->err.clear();
    return fail(ctx, LRS_EINVAL, "omega must be finite and >= 0");
  }
  return make_quadrature(ctx, LRS_QUAD_TIME, nnodes, scale, omega);
}

static lrs_status make_quadrature(lrs_ctx* ctx, int kind, int nnodes, double scale,
                                  double omega) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (ctx->graph_pinned)
    return fail(ctx, LRS_ESTATE, "captured graphs read this context's buffers; call "
                "lrs_release_graphs once those graphs are gone");
  if (!ctx->have_bands) return fail(ctx, LRS_ESTATE, "lrs_set_orbitals must come first");
  if (kind != LRS_QUAD_TIME && kind != LRS_QUAD_FREQ) return fail(ctx, LRS_EINVAL, "unknown quadrature kind %d", kind);
  if (nnodes < 1 || nnodes > 64) return fail(ctx, LRS_EINVAL, "nnodes must be 1..64");
  if (!std::isfinite(scale)) return fail(ctx, LRS_ENONFINITE, "non-finite scale");
  std::vector<double> x, y;
  offsets(ctx, x, y);
  std::vector<double> a, wgl;
  gauss_legendre_01(nnodes, a, wgl);
  const int Ko = ctx->Ko, Ku = ctx->Ku;
  Quad q;
  q.kind = kind;
  std::vector<double> c, ci, al, be, dal, dbe;
  // derivative of an offset with respect to its band energy (mu fixed):
  // x = mu - e -> -1, y = e - mu -> +1, times x/sqrt(x^2+delta^2) with regularisation
  auto dx_de = [&](double xr, double sign) {
    if (ctx->delta > 0) return sign * (xr / std::sqrt(xr * xr + ctx->delta * ctx->delta));
    return sign;
  };
  std::vector<double> xr(Ko), yr(Ku);   // unregularised offsets
  for (int k = 0; k < ctx->nk; ++k) {
    for (int n = 0; n < ctx->nocc; ++n) xr[(size_t)k * ctx->nocc + n] = ctx->mu - ctx->energies[(size_t)k * ctx->nb + n];
    for (int m = 0; m < ctx->nu; ++m) yr[(size_t)k * ctx->nu + m] = ctx->energies[(size_t)k * ctx->nb + ctx->nocc + m] - ctx->mu;
  }
  if (kind == LRS_QUAD_TIME) {
    double dmin = *std::min_element(x.begin(), x.end()) + *std::min_element(y.begin(), y.end());
    double dmax = *std::max_element(x.begin(), x.end()) + *std::max_element(y.begin(), y.end());
    if (!(dmin > 0)) return fail(ctx, LRS_ENOGAP, "smallest denominator is not positive");
    double C = scale > 0 ? scale : time_auto_scale_iw(dmin, dmax, nnodes, omega);
    q.scale = C;
    q.omega = omega;
    for (int j = 0; j < nnodes; ++j) {
      double tau = C * a[j] / (1.0 - a[j]);
      double cj = C * wgl[j] / ((1.0 - a[j]) * (1.0 - a[j]));
      // imaginary frequency: complex coefficient c e^{i omega tau} (Laplace transform of
      // cos and sin); omega = 0 leaves the static rule
      if (omega != 0.0) ci.push_back(cj * std::sin(omega * tau));
      c.push_back(omega != 0.0 ? cj * std::cos(omega * tau) : cj);
      q.tau.push_back(tau);
      for (int i = 0; i < Ko; ++i) {
        double v = std::exp(-x[i] * tau);
        al.push_back(v);
        dal.push_back(-tau * v * dx_de(xr[i], -1.0));
      }
      for (int i = 0; i < Ku; ++i) {
        double v = std::exp(-y[i] * tau);
        be.push_back(v);
        dbe.push_back(-tau * v * dx_de(yr[i], 1.0));
      }
    }
  } else {
    double zeta = scale;
    if (!(scale > 0)) {
      double lo = INFINITY, hi = 0;
      for (double e : ctx->energies) {
        double d = std::fabs(ctx->mu - e);
        lo = std::min(lo, d);
        hi = std::max(hi, d);
      }
      if (ctx->delta > 0) {
        double f = 0.5 / kHartreeEv;
        lo = std::sqrt(lo * lo + f * f);
      }
      zeta = std::sqrt(lo * hi);
    }
    q.scale = zeta;
    for (int part = 0; part < 2; ++part) {      // p-terms, then q-terms
      for (int j = 0; j < nnodes; ++j) {
        double t = zeta * a[j] / (1.0 - a[j]);
        double cj = zeta * wgl[j] / (kPi * (1.0 - a[j]) * (1.0 - a[j]));
        c.push_back(cj);
        q.tau.push_back(t);
        auto f = [&](double v) { return part == 0 ? v / (v * v + t * t) : t / (v * v + t * t); };
        auto df = [&](double v) {   // derivative with respect to the offset v
          double d = v * v + t * t;
          return part == 0 ? (t * t - v * v) / (d * d) : -2.0 * v * t / (d * d);
        };
        for (int i = 0; i < Ko; ++i) {
          al.push_back(f(x[i]));
          dal.push_back(df(x[i]) * dx_de(xr[i], -1.0));
        }
        for (int i = 0; i < Ku; ++i) {
          be.push_back(f(y[i]));
          dbe.push_back(df(y[i]) * dx_de(yr[i], 1.0));
        }
      }
    }
  }
  if ((int)c.size() > kMaxTerms) return fail(ctx, LRS_EINVAL, "too many terms");
  drop_quad(ctx);
  CHECK(install_terms(ctx, q, c, al, be, &dal, &dbe, ci.empty() ? nullptr : &ci));
  ctx->quad = q;
  return LRS_OK;
}

lrs_status lrs_make_quadrature_tol(lrs_ctx* ctx, double tol, int nmin, int nmax, int* nnodes_host,
                                   double* err_host) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (!ctx->have_bands) return fail(ctx, LRS_ESTATE, "lrs_set_orbitals must come first");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, LRS_EINVAL, "tol must be finite and > 0");
  if (nmin < 1 || nmax > 64 || nmin > nmax) return fail(ctx, LRS_EINVAL, "need 1 <= nmin <= nmax <= 64");
  std::vector<double> x, y;
  offsets(ctx, x, y);
  const double dmin = *std::min_element(x.begin(), x.end()) + *std::min_element(y.begin(), y.end());
  const double dmax = *std::max_element(x.begin(), x.end()) + *std::max_element(y.begin(), y.end());
  if (!(dmin > 0)) return fail(ctx, LRS_ENOGAP, "smallest denominator is not positive");
  // the smallest node count whose rule (at its own best scale) meets tol on every gap in
  // [dmin, dmax]; the band-energy range alone decides it
  int n = nmax;
  double C = 0, e = 0;
  for (int m = nmin; m <= nmax; ++m) {
    C = time_auto_scale(dmin, dmax, m);
    e = time_rule_error(C, m, dmin, dmax);
    if (e <= tol) {
      n = m;
      break;
    }
  }
  CHECK(make_quadrature(ctx, LRS_QUAD_TIME, n, C, 0.0));
  if (nnodes_host) *nnodes_host = n;
  if (err_host) *err_host = e;
  return LRS_OK;
}

lrs_status lrs_get_quadrature(const lrs_ctx* ctx, int* nterms, double* c_host, double* tau_host,
                              double* mu_host, double* scale_host) {
  if (!ctx || !nterms) return LRS_EINVAL;
  if (!ctx->have_quad) return LRS_ESTATE;
  *nterms = ctx->quad.nterms;
  // report the caller-facing coefficients: undo the per-term power-of-two normalisation
  if (c_host || tau_host) {
    for (int t = 0; t < ctx->quad.nterms; ++t) {
      if (c_host) c_host[t] = ctx->quad.c_raw.empty() ? ctx->quad.c[t] : ctx->quad.c_raw[t];
      if (tau_host) tau_host[t] = ctx->quad.tau[t];
    }
  }
  if (mu_host) *mu_host = ctx->mu;
  if (scale_host) *scale_host = ctx->quad.scale;
  return LRS_OK;
}

lrs_status lrs_compute_chi0(lrs_ctx* ctx, int site, int cols, int prec, double* out) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (!ctx->have_bands || !ctx->have_sites || !ctx->have_quad)
    return fail(ctx, LRS_ESTATE, "orbitals, sites and quadrature must be set first");
  if (!out) return fail(ctx, LRS_EINVAL, "chi0_out is NULL");
  if (site < -1 || site >= ctx->nsites) return fail(ctx, LRS_EINVAL, "site %d out of range", site);
  if (cols != LRS_COLS_GRID && cols != LRS_COLS_SITE) return fail(ctx, LRS_EINVAL, "bad column set");
  if (prec < LRS_FP64 || prec > LRS_FP64_3M) return fail(ctx, LRS_EINVAL, "bad precision");
  if (ctx->real_mode && prec != LRS_FP64 && prec != LRS_F16F8)
    return fail(ctx, LRS_EUNSUPPORTED, "real orbitals: LRS_FP64 or LRS_F16F8 only");
  if (cols == LRS_COLS_GRID && ctx->ngrid <= 0) return fail(ctx, LRS_ESTATE, "no grid orbitals were given");
  int cur = -1;
  HIP_OR_FAIL(ctx, hipGetDevice(&cur));
  if (cur != ctx->device) HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  // under stream capture the call records its kernels only: no timing events, and anything
  // that would allocate or build a plan is refused
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_OR_FAIL(ctx, hipStreamIsCapturing(ctx->stream, &cs));
  ctx->capturing = cs != hipStreamCaptureStatusNone;
  if (ctx->capturing) ctx->timed = false;
  const lrs_status st = run_chi0(ctx, site, cols, prec, pick_variant(ctx, prec, cols), out, !ctx->capturing);
  // a captured call bakes the context's buffers into the graph: keep them in place.  The site
  // operand it recorded was not built yet, so the kept one describes nothing.
  if (ctx->capturing) {
    if (st == LRS_OK) ctx->graph_pinned = true;
    ctx->a_prec = -1;
  }
  ctx->capturing = false;
  return st;
}

lrs_status lrs_release_graphs(lrs_ctx* ctx) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  ctx->graph_pinned = false;
  ctx->a_prec = -1;        // replays may have rewritten the site operand
  return LRS_OK;
}

double lrs_last_kernel_ms(lrs_ctx* ctx) {
  if (!ctx || !ctx->timed) return -1.0;
  float ms = -1.f;
  if (hipEventSynchronize(ctx->ev1) != hipSuccess || hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) != hipSuccess)
    return -1.0;
  return ms;
}

// The tuner times every compiled variant of precision prec on each column set of the current
// problem (the cell grid if it was given, and the site blocks), on the site with the most
// points (the shape class that dominates the launch): the site x grid launch over its first
// two rounds of tiles of the real plan (XCD meeting included), the site block whole.  The score
// is milliseconds per output entry actually covered, so tile shapes of different size and
// raggedness compare fairly; each sample runs once to warm up and twice timed (the faster
// counts).  The choice is kept per (precision, column set) for later lrs_compute_chi0 calls and
// appended to the file named by LRS_TUNE_CACHE, keyed by precision, column set and problem
// shape (rows of that site, columns, K, terms).
lrs_status lrs_tune(lrs_ctx* ctx, int prec) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (!ctx->have_bands || !ctx->have_sites || !ctx->have_quad)
    return fail(ctx, LRS_ESTATE, "orbitals, sites and quadrature must be set first");
  if (prec < LRS_FP64 || prec > LRS_FP64_3M) return fail(ctx, LRS_EINVAL, "bad precision");
  if (ctx->real_mode && prec != LRS_FP64 && prec != LRS_F16F8)
    return fail(ctx, LRS_EUNSUPPORTED, "real orbitals: LRS_FP64 or LRS_F16F8 only");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  int s = 0;
  for (int k = 1; k < ctx->nsites; ++k)
    if (ctx->site_off[k + 1] - ctx->site_off[k] > ctx->site_off[s + 1] - ctx->site_off[s]) s = k;
  const int nr = ctx->site_off[s + 1] - ctx->site_off[s];
  const char* path = std::getenv("LRS_TUNE_CACHE");
  for (int cols = LRS_COLS_GRID; cols <= LRS_COLS_SITE; ++cols) {
    if (cols == LRS_COLS_GRID && ctx->ngrid <= 0) continue;
    std::ostringstream key;
    key << "prec=" << prec << " cols=" << cols << " rows=" << nr
        << " ncols=" << (cols == LRS_COLS_GRID ? ctx->ngrid : nr) << " K=" << ctx->K_pad
        << " T=" << ctx->quad.nterms << " iw=" << (ctx->quad.ci.empty() ? 0 : 1);
    bool cached = false;
    if (path) {
      std::ifstream in(path);
      std::string line;
      while (std::getline(in, line)) {
        const size_t p = line.rfind(" variant=");
        if (p != std::string::npos && line.substr(0, p) == key.str()) {
          const int v = std::atoi(line.c_str() + p + 9);
          if (v >= 0 && v < chi0_num_variants(prec)) {
            ctx->tuned_variant[prec][cols] = v;
            cached = true;
          }
        }
      }
    }
    if (cached) continue;
    const long long ncol = cols == LRS_COLS_GRID ? ctx->ngrid : nr;
    DevBuf out;
    CHECK(ensure_buf(ctx, out, (size_t)nr * ncol * 8, "tuning output"));
    int best = chi0_default_variant(prec);
    double best_score = HUGE_VAL;
    for (int v = 0; v < chi0_num_variants(prec); ++v) {
      Plan* plan = nullptr;
      const bool odd = !ctx->quad.ci.empty();
      lrs_status st = get_plan(ctx, s, cols, prec, v, cols == LRS_COLS_SITE && odd ? 2 : 0, &plan);
      if (st != LRS_OK) { release(ctx, out); return st; }
      const Batch& b0 = plan->batches[0];
      const int sample = cols == LRS_COLS_GRID ? std::min(b0.ntiles, 2 * b0.grid) : 0;
      const long long area = sample > 0 ? plan->area[b0.tile0 + sample] - plan->area[b0.tile0]
                                        : plan->area.back();
      float ms = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev0, ctx->stream));
        st = run_chi0(ctx, s, cols, prec, v, (double*)out.p, false, sample);
        if (st != LRS_OK) { release(ctx, out); return st; }
        HIP_OR_FAIL(ctx, hipEventRecord(ctx->ev1, ctx->stream));
        HIP_OR_FAIL(ctx, hipEventSynchronize(ctx->ev1));
        float t = 0;
        HIP_OR_FAIL(ctx, hipEventElapsedTime(&t, ctx->ev0, ctx->ev1));
        if (rep > 0) ms = std::min(ms, t);
      }
      const double score = ms / (double)std::max<long long>(area, 1);
      if (score < best_score) {
        best_score = score;
        best = v;
      }
    }
    release(ctx, out);
    ctx->tuned_variant[prec][cols] = best;
    if (path) {
      std::ofstream o(path, std::ios::app);
      o << key.str() << " variant=" << best << "\n";
    }
  }
  ctx->timed = false;
  return LRS_OK;
}

lrs_status lrs_tuned_variant(const lrs_ctx* ctx, int prec, int cols, int* variant_host,
                             int* tile_rows_host, int* tile_cols_host) {
  if (!ctx || !variant_host) return LRS_EINVAL;
  if (prec < LRS_FP64 || prec > LRS_FP64_3M || (cols != LRS_COLS_GRID && cols != LRS_COLS_SITE))
    return LRS_EINVAL;
  const int v = pick_variant(const_cast<lrs_ctx*>(ctx), prec, cols);
  *variant_host = v;
  const TileShape sh = chi0_shape(prec, v);
  if (tile_rows_host) *tile_rows_host = sh.bm;
  if (tile_cols_host) *tile_cols_host = sh.bn;
  return LRS_OK;
}

lrs_status lrs_screen_W(lrs_ctx* ctx, const double* chi0_ss, double* W_out, const double* rho,
                        double* loss_out) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (!ctx->have_sites) return fail(ctx, LRS_ESTATE, "sites must be set first");
  if (!chi0_ss || !W_out) return fail(ctx, LRS_EINVAL, "chi0 and W_out are required");
  if (loss_out && !rho) return fail(ctx, LRS_EINVAL, "loss_out needs rho_test");
  if (!screen_sizes_ok(ctx))
    return fail(ctx, LRS_EUNSUPPORTED, "a site basis exceeds 448 functions or 256 directions");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipError_t e = launch_screen_forward(ctx, chi0_ss, W_out, rho, loss_out);
  if (e == hipErrorOutOfMemory) return fail(ctx, LRS_ENOMEM, "screening workspace");
  if (e != hipSuccess) return fail(ctx, LRS_EDEVICE, "screen_W: %s", hipGetErrorString(e));
  return LRS_OK;
}

lrs_status lrs_screen_W_backward(lrs_ctx* ctx, const double* dL_dW, double* dL_dchi0) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (!ctx->have_W) return fail(ctx, LRS_ESTATE, "lrs_screen_W must come first");
  if (!dL_dchi0) return fail(ctx, LRS_EINVAL, "dL_dchi0 is required");
  if (!dL_dW && !ctx->have_rho) return fail(ctx, LRS_EINVAL, "dL_dW is NULL and no test charge was given");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipError_t e = launch_screen_backward(ctx, dL_dW, dL_dchi0);
  if (e != hipSuccess) return fail(ctx, LRS_EDEVICE, "screen_W backward: %s", hipGetErrorString(e));
  return LRS_OK;
}

lrs_status lrs_compute_chi0_backward(lrs_ctx* ctx, int cols, int prec, const double* dL_dchi0,
                                     double* dL_dE, void* dL_dpsi_site, void* dL_dpsi_grid) {
  if (!ctx) return LRS_EINVAL;
  ctx->err.clear();
  if (!ctx->have_bands || !ctx->have_sites || !ctx->have_quad)
    return fail(ctx, LRS_ESTATE, "orbitals, sites and quadrature must be set first");
  if (cols != LRS_COLS_SITE) return fail(ctx, LRS_EUNSUPPORTED, "backward supports site x site blocks only");
  if (prec != LRS_FP64 && prec != LRS_BF16X2 && prec != LRS_F16F8)
    return fail(ctx, LRS_EUNSUPPORTED, "backward precision must be LRS_FP64, LRS_BF16X2 or "
                "LRS_F16F8");
  if (dL_dpsi_grid) return fail(ctx, LRS_EUNSUPPORTED, "site blocks do not depend on grid orbitals");
  if (ctx->real_mode && (prec != LRS_F16F8 || ctx->g_keep_prec != LRS_F16F8))
    return fail(ctx, LRS_EUNSUPPORTED, "real orbitals: the adjoint runs in LRS_F16F8 from the "
                "Green's functions an LRS_F16F8 chi0 call over every site block keeps (none kept "
                "for the current terms)");
  if (!dL_dchi0 || !dL_dE || !dL_dpsi_site) return fail(ctx, LRS_EINVAL, "missing gradient buffers");
  if (!ctx->quad.has_deriv) return fail(ctx, LRS_EUNSUPPORTED, "generic terms carry no energy derivative");
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_OR_FAIL(ctx, hipStreamIsCapturing(ctx->stream, &cs));
  if (cs != hipStreamCaptureStatusNone)
    return fail(ctx, LRS_ESTATE, "the backward pass copies host tables and synchronises; it "
                "cannot be captured");
  hipError_t e = launch_chi0_backward(ctx, prec, dL_dchi0, dL_dE, (double*)dL_dpsi_site);
  if (e == hipErrorIllegalState) return LRS_ESTATE;   // message set by the refused buffer
  if (e == hipErrorOutOfMemory) return fail(ctx, LRS_ENOMEM, "adjoint workspace");
  if (e != hipSuccess) return fail(ctx, LRS_EDEVICE, "chi0 backward: %s", hipGetErrorString(e));
  return LRS_OK;
}

}  // extern "C"
