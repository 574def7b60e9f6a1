// Internal declarations of the screening library: context state, operand layouts and
// kernel launchers.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/lrs.h"

namespace lrs {

// Operand chunking along K (the flattened (k-point, band) index).  A "fragment tile" is
// 16 rows (or columns) x one K chunk of a precision's matrix-core operand, every lane's operand
// contiguous: FP64 -> 16 k x 2 planes (re, im) x 8 B = 4 KiB; FP32 -> 32 k x 2 planes x 4 B
// = 4 KiB; BF16X2/FP16X2 -> 16 k x 4 planes (re hi, re lo, im hi, im lo) x 2 B = 2 KiB.
// Operands are stored chunk-major ([chunk][block][tile]).
constexpr int kTileBytes = 4096;   // FP64 and FP32 tiles
constexpr int kChunkF64 = 16;
constexpr int kRowAlign = 128;  // rows / columns of every operand are padded to this
// widest output tile of any kernel variant: column operands carry this much slack past their
// last 128-column slot, so a full-width last tile reads inside the operand
constexpr int kMaxTileCols = 256;
// each K phase (occupied, unoccupied) is padded to this: a multiple of four chunks of every
// precision, so the kernel's four-slot LDS ring starts every phase at slot 0
constexpr int kPhaseAlign = 128;
// largest set of Green's functions an F16F8, BF16X2 or FP64 site-block launch keeps for the
// adjoint
constexpr size_t kKeepMaxBytes = (size_t)16 << 30;
constexpr int kMaxTerms = 128;

__host__ __device__ inline bool is_split(int prec) { return prec == LRS_BF16X2 || prec == LRS_FP16X2; }
// operands carry fp16 values prescaled by a power of two (FP16X2 and F16F8)
__host__ __device__ inline bool is_f16(int prec) { return prec == LRS_FP16X2 || prec == LRS_F16F8; }
constexpr int kNumPrec = 6;
// leading dimension of a site's n x n block: n for chi0 outputs, n rounded up to kAdjAlign for
// the adjoint's internal site blocks (plan mode 1): a whole number of four-chunk ring cycles
// of the adjoint GEMMs' contraction, whose padding is zero
constexpr int kAdjAlign = 64;
__host__ __device__ inline int site_block_ld(int n, int mode) {
  return mode == 1 ? (n + kAdjAlign - 1) / kAdjAlign * kAdjAlign : n;
}
// K values per chunk and bytes per fragment tile (16 rows x chunk x planes)
__host__ __device__ inline int chunk_of(int prec) { return prec == LRS_FP32 ? 32 : 16; }
__host__ __device__ inline int tile_bytes(int prec) {
  return is_split(prec) || prec == LRS_F16F8 ? 2048 : (prec == LRS_FP64_3M ? 6144 : 4096);
}
// F16F8 fragment tiles (16 rows x 16 K, 2 KiB; a 32-row block is two consecutive tiles):
//   [0, 1024)    fp16 hi: planes re, im, 512 B each, slot s holding row s%16 and
//                K 8 (s/16) + e, e = 0..7 (16 B)
//   [1024, 2048) fp8 (e4m3) planes re part 0, re part 1, im part 0, im part 1, 256 B each,
//                row r at 16 r holding K 0..15 (16 B).  The fp8 fragment of a lane is one
//                component's part 0 (its scale block 0 of the matrix-core instruction) and
//                part 1 (block 1): re in lanes 0-31, im in lanes 32-63, so that one instruction
//                takes the cross terms of both products of a complex multiply-add.  The row
//                (site) operand stores hi * 2^7 in part 0 and lo * 2^18 in part 1; the column
//                operand the other way round, so that the blocks multiply hi * lo and lo * hi.
constexpr int kF8HiShift = 7;    // fp8 hi = e4m3(hi * 2^7): |hi| < 2 after the prescale
constexpr int kF8LoShift = 18;   // fp8 lo = e4m3(lo * 2^18): |lo| <= 2^-11 |x| < 2^-10

// x to fp8 e4m3 (1 sign, 4 exponent bits with bias 7, 3 mantissa bits; no infinities, the
// largest finite value 448), rounding to nearest with ties to even; values beyond 448 saturate
// to it.  Below 2^-6 the format is subnormal (steps of 2^-9).
__device__ inline unsigned int e4m3_rn(float x) {
  const unsigned int sign = (__float_as_uint(x) >> 24) & 0x80u;
  const float a = fabsf(x);
  if (a < 0.015625f) return sign | (unsigned int)rintf(a * 512.0f);   // 8 -> 0x08 = 2^-6
  unsigned int u = __float_as_uint(a);
  u += 0x7FFFFu + ((u >> 20) & 1u);                  // round the mantissa to 3 bits
  const int e = (int)(u >> 23) - 120;                // rebias 127 -> 7
  const unsigned int m = (u >> 20) & 7u;
  if (e > 15 || (e == 15 && m == 7)) return sign | 0x7Eu;
  return sign | ((unsigned int)e << 3) | m;
}
inline long long round_up(long long x, long long m) { return (x + m - 1) / m * m; }
// Split adjoint operand tiles (bfloat16).  A 1 KiB piece holds 32 rows x 16 contraction
// indices of one plane, lane l's 16 bytes at 16 l being row l%32, indices 8 (l/32) .. +7; the
// four planes (re hi, re lo, im hi, im lo) of a piece follow each other (4 KiB groups), and
// groups go contraction-chunk-major.  Element offset of (row p, index r) in a site block of
// H (ld = the block's padded size, a multiple of 64), plane 0:
__host__ __device__ inline long long h_tile_offset(int p, int r, int ld) {
  return (((long long)(r >> 4) * (ld >> 5) + (p >> 5)) << 11) +
         (((p & 31) + ((r >> 3) & 1) * 32) << 3) + (r & 7);
}

// One output tile of a chi0 launch.
struct TileDesc {
  int a_row0;           // first row of the site operand
  int b_col0;           // first column of the column operand (multiple of 16)
  int nrows;            // valid rows in this tile
  int ncols;            // valid columns
  long long out_off;    // element offset of the tile's (0,0) in the output
  int ldo;              // output leading dimension
  int pad;              // site blocks: first site row - first site column (else 0)
  int m0, c0;           // site blocks: first row and first column within the block (else 0)
};
static_assert(sizeof(TileDesc) == 40, "TileDesc layout");

// Tile shape of one kernel instantiation.
struct TileShape {
  int bm, bn;           // workgroup tile
  int threads;
  size_t park_bytes;    // per-workgroup scratch for G_o
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Batch {            // a contiguous range of site row blocks and its tiles
  int rb0 = 0, nrb = 0;   // row blocks (16 slot rows each) of the weighted site operand
  int tile0 = 0, ntiles = 0;
  int grid = 0;
};

struct Plan {             // cached launch plan for (site, cols, prec, variant, mode)
  DevBuf tiles;
  std::vector<long long> area;   // output entries covered by the first i tiles (prefix sums)
  int ntiles = 0;
  int variant = 0;
  std::vector<Batch> batches;
};

struct Quad {
  int kind = -1;          // LRS_QUAD_TIME, LRS_QUAD_FREQ, or -1 generic
  int nterms = 0;
  double scale = 0;       // C (time) or zeta (freq)
  std::vector<double> c;        // per-term coefficient after weight normalisation
  std::vector<double> c_raw;    // per-term coefficient as constructed
  std::vector<double> ci;       // imaginary parts after normalisation (imaginary frequency)
  double omega = 0;             // imaginary frequency of the rule (0: static)
  std::vector<double> tau;      // tau (time) or t (freq) per term
  std::vector<double> w;        // [T][K_pad] normalised alpha | beta (zero padded)
  std::vector<double> dw;       // [T][K_pad] d(weight)/d(energy) with mu fixed
  // real orbitals: w and dw hold the slot layout; these the orbital order [T][2 K_pad]
  std::vector<double> w_orb, dw_orb;
  bool has_deriv = false;
};

}  // namespace lrs

struct lrs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  std::string err;
  size_t bytes_in_use = 0;
  size_t max_bytes = 0;   // 0 = unlimited

  // bands
  bool have_bands = false;
  int nk = 0, nb = 0, nocc = 0, nu = 0, spin = 2;
  double mu = 0, delta = 0;
  std::vector<double> energies;   // [nk][nb]
  int ngrid = 0;
  double grid_dV = 0;
  // K layout: [0, Ko) occupied (k-major), zeros to Ko_pad, then [Ko_pad, Ko_pad+Ku) unoccupied
  int Ko = 0, Ku = 0, Ko_pad = 0, Ku_pad = 0, K_pad = 0;
  // real orbitals at one k (lrs_set_orbitals_real): Ko and Ku count orbitals, Ko_pad, Ku_pad
  // and K_pad count operand slots, two orbitals each
  bool real_mode = false;

  // grid operand: FP64 fragment tiles (always) and lazily built reduced-precision tiles
  lrs::DevBuf grid_tiles[lrs::kNumPrec];
  int grid_cols_pad = 0;
  float grid_scale_f16 = 1.f;     // power-of-two prescale used by the FP16X2 and F16F8 tiles

  // sites
  bool have_sites = false;
  int nsites = 0, lmax = 2, nrows = 0, rows_pad = 0;
  std::vector<int> nrad, nang, site_off, rad_off, ang_off;
  std::vector<int> site_col_off;  // column offset of each site in the site column operand
  int site_cols_pad = 0;
  float site_scale_f16 = 1.f;     // power-of-two prescale of site values in FP16X2 and F16F8 operands
  lrs::DevBuf site_colmap;        // [site_cols_pad] column -> site row (-1: zero column)
  std::vector<double> radii, rad_w, ang_xyz, ang_w;
  lrs::DevBuf site_f64;           // planar re/im [2][rows_pad][K_pad] (chunk-permuted), FP64
  lrs::DevBuf site_tiles[lrs::kNumPrec];   // site points as a column operand (fragment tiles)
  lrs::DevBuf a_tiles;            // weighted site operand tiles of the current batch
  lrs::DevBuf park;               // per-workgroup G_o scratch of the chi0 launches
  // Green's functions of every term on the site blocks, kept by an F16F8, BF16X2 or FP64 chi0
  // launch over all sites for the adjoint (G_o then G_u, complex [T][sum n^2] each: FP64 for
  // the FP64 path, else FP32); g_keep_prec is the precision they hold, -1 when absent or stale
  lrs::DevBuf g_keep;
  int g_keep_prec = -1;
  lrs::DevBuf xcd_sync;           // per-XCD term counters of the chi0 launches
  int a_prec = -1, a_version = -1, a_rb0 = -1, a_nrb = -1, a_t0 = -1, a_nt = -1;
  lrs::DevBuf psi_site_f64;       // planar [2][K_pad][rows_pad] (k-major rows) for the adjoint
  lrs::DevBuf psi_site_bf16;      // the same split: bfloat16 [4][K_pad][rows_pad] (re hi, re lo,
                                  // im hi, im lo) for the split adjoint
  bool psi_kmajor_ok = false, psi_split_ok = false;   // the two above are current
  float site_max_abs = 0.f;
  float grid_max_abs = 0.f;

  // quadrature
  bool have_quad = false;
  lrs::Quad quad;
  lrs::DevBuf w_nat, c_dev;       // weights [T][K_pad] (natural K order), coefficients [T]
                                  // (then their imaginary parts [T] when the rule has them)
  int quad_version = 0;

  // plans
  std::map<long long, lrs::Plan> plans;
  // variant chosen by lrs_tune per (precision, column set); -1 = the default
  int tuned_variant[lrs::kNumPrec][2] = {{-1, -1}, {-1, -1}, {-1, -1}, {-1, -1}, {-1, -1},
                                         {-1, -1}};

  // screening state
  lrs::DevBuf W_last, rho_last, screen_tab, work, adj_work, val_work, fft_work;
  lrs::DevBuf probe;              // output of the matrix-core rate probe
  lrs::DevBuf proj_work;          // workspace of the direct projection
  bool have_W = false, have_rho = false;

  // timing
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  // set while a call runs on a stream that is being captured into a graph: nothing may
  // allocate, copy from the host or synchronise then
  bool capturing = false;
  // set once a call has been captured: graphs then hold this context's buffer addresses, so
  // calls that would free or replace those buffers are refused until lrs_release_graphs
  bool graph_pinned = false;
};

namespace lrs {

// quadrature.cpp
void gauss_legendre_01(int n, std::vector<double>& a, std::vector<double>& w);
double time_rule_error(double scale, int n, double dmin, double dmax);
double time_auto_scale(double dmin, double dmax, int n);
double time_auto_scale_iw(double dmin, double dmax, int n, double omega);

// pack.hip
// real != 0: one k of real orbitals (the real parts of psi), two to a slot (Ko_pad and K_pad
// count slots)
hipError_t launch_pack_tiles(const double* psi, int nk, int nb, int nocc, int ncols, int ld_src,
                             int ncols_pad, int Ko_pad, int K_pad, int prec, float prescale,
                             int real, void* out, hipStream_t s);
hipError_t launch_pack_site_rows(const double* psi, int nk, int nb, int nocc, int nrows,
                                 int rows_pad, int Ko_pad, int K_pad, int real, double* out_f64,
                                 hipStream_t s);
// largest |Im psi| over n complex values, as float bits (0 if all vanish)
hipError_t launch_max_abs_im(const double* psi, long long n, unsigned int* out_bits,
                             hipStream_t s);
// planar [2][K][rows_pad] site orbitals in natural K order from the FP64 row operand; real: the
// operand holds two real orbitals per slot, and out gets the 2 K_pad orbitals with zero
// imaginary parts
hipError_t launch_derive_site_kmajor(const double* site_f64, int rows_pad, int K_pad, int real,
                                     double* out, hipStream_t s);
hipError_t launch_site_col_tiles(const double* site_f64, int rows_pad, int K_pad, int ncols_pad,
                                 const int* colmap, int prec, float prescale, void* dst,
                                 hipStream_t s);
hipError_t launch_max_abs(const double* x, long long n, unsigned int* out_bits, hipStream_t s);
hipError_t launch_repack_from_f64(const void* tiles64, int ncols_pad, int K_pad, int prec,
                                  float prescale, void* dst, hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);

// chi0.hip
int chi0_num_variants(int prec);
int chi0_blocks_per_cu(int prec, int variant);
int chi0_default_variant(int prec);
TileShape chi0_shape(int prec, int variant);
// the variant keeps its B fragments rotating through registers (split paths): its products
// reach each element in another order than the other variants'
bool chi0_variant_rotates(int prec, int variant);
// w: weights [T][w_stride]; a slot's im-plane value takes the weight at q_woff + k (0 for
// complex orbitals; K_pad for real orbitals, whose second orbital of a slot has its own)
hipError_t launch_prep_site(int prec, const double* site, int rows_pad, int K_pad,
                            const int* slot_row, int rb0, int nrb, const double* w,
                            int w_stride, int q_woff, int t0, int nt, double a_scale, void* out,
                            hipStream_t s);
// sym: site x site blocks, listed from their upper triangle (TileDesc.pad set): each element
// on or above the diagonal is also stored at its transposed place
// ci: imaginary parts of the term coefficients (null: real); sym must be 0 then (the odd
// part of chi0 at imaginary frequency is antisymmetric on a site block)
// real: the operands hold real orbitals two to a slot (FP64 and F16F8 only)
// keep_o, keep_u (site blocks, or null): each term's G_o and G_u as complex (FP64 for the FP64
// paths, else FP32) at the output's element offsets plus t * keep_stride, on and above the
// diagonal
hipError_t launch_chi0(int prec, int variant, int grid, const void* a_tiles, int a_nrb,
                       const void* b_tiles, int b_ncb, int nch, const double* c,
                       const double* ci, int T, int nch_o, const TileDesc* tiles, int ntiles,
                       double* out, double pref, int sym, unsigned int* sync, void* park,
                       int real, void* keep_o, void* keep_u, long long keep_stride,
                       hipStream_t s);
// adjoint Green's functions of one term on site blocks: prec LRS_FP64 writes Hu, Ho as FP64
// planes (hu_re, hu_im, ho_re, ho_im; row stride ld); LRS_BF16X2 and LRS_F16F8 (variant 1)
// write each at hs_u, hs_o as bfloat16 hi/lo in the split adjoint GEMM's operand tiles
// (h_tile_offset)
hipError_t launch_green_adjoint(int prec, int grid, const void* a_tiles, int a_nrb,
                                const void* b_tiles, int b_ncb, int nch, const double* c,
                                int nch_o, const TileDesc* tiles, int ntiles, const double* lam,
                                const double* lam_a, double adj_c, double adj_s,
                                double* hu_re, double* hu_im, double* ho_re, double* ho_im,
                                void* hs_u, void* hs_o, void* park, hipStream_t s);
// the same split H (hs_u, hs_o) of one term from its kept G_o, G_u (keep_o, keep_u at the
// caller's site-block offsets blk_off; lam, lam_a and H at the padded offsets pblk_off;
// blk_n on the device, blk_n_host its host copy)
// the FP64 H planes (hu_re, hu_im, ho_re, ho_im, padded row stride) of one term from its kept
// FP64 G_o, G_u, as the mode-1 epilogue writes them
hipError_t launch_h_from_kept_f64(const void* keep_o, const void* keep_u, int nsites,
                                  const long long* blk_off, const long long* pblk_off,
                                  const int* blk_n, const double* lam, const double* lam_a,
                                  double adj_c, double adj_s, double* hu_re, double* hu_im,
                                  double* ho_re, double* ho_im, hipStream_t s);
hipError_t launch_h_from_kept(const void* keep_o, const void* keep_u, int nsites,
                              const long long* blk_off, const long long* pblk_off,
                              const int* blk_n, const int* blk_n_host, const double* lam,
                              const double* lam_a,
                              double adj_c, double adj_s, void* hs_u, void* hs_o,
                              hipStream_t s);

// lrs_api.cpp (shared with the adjoint)
lrs_status plan_for(lrs_ctx* ctx, int site, int cols, int prec, int variant, int mode,
                    Plan** out);
lrs_status ensure_site_tiles_for(lrs_ctx* ctx, int prec);
// weighted site operand of terms [t0, t0 + nt) for batch b's rows; *a = the first term's part
lrs_status ensure_site_operand(lrs_ctx* ctx, int prec, const Batch& b, int t0, int nt,
                               const void** a);
lrs_status ensure_park(lrs_ctx* ctx, int prec, int variant, int grid);

// screen.hip
// size of the fixed device array that holds the tables and workspace of lrs_screen_W_noalloc
constexpr size_t kScratchBytes = (size_t)64 << 20;
// the per-site solves' limits: basis functions n = (lmax + 1)^2 n_rad (49 shells at lmax 2) and
// directions per shell
constexpr int kMaxBasis = 448, kMaxDirections = 256;
hipError_t scratch_setup(int device);
bool screen_sizes_ok(const lrs_ctx* ctx);
hipError_t launch_screen_forward(lrs_ctx* ctx, const double* chi0_ss, double* W_out,
                                 const double* rho, double* loss_out);
hipError_t launch_screen_backward(lrs_ctx* ctx, const double* dL_dW, double* dL_dchi0);

// adjoint.hip
hipError_t launch_chi0_backward(lrs_ctx* ctx, int prec, const double* dL_dchi0, double* dL_dE,
                                double* dL_dpsi);

}  // namespace lrs
