// Main loop of a complex FP64 GEMM workgroup tile, shared by the adjoint's Y = H psi and the
// orbital projection psi = C P^T (included by HIP sources only).
//
// Y[m][n] += sum_k A[m][k] B[n][k] over complex values held as separate real and imaginary
// planes, each operand row contiguous along k.  64 x 128 workgroup tiles from 2 x 2 waves of
// 32 x 64 (2 x 4 blocks of v_mfma_f64_16x16x4).  The contraction order is free, so lane l of
// matrix-core step s takes k = 4 (l/16) + s: its four values of a 16-wide chunk are then four
// consecutive k of one operand row, and each lane's 32 bytes per plane come straight from the
// natural layout as two 16-byte direct-to-LDS loads.  A 16-row (or 16-column) tile of a chunk
// takes 4 KiB of LDS, [plane][half][lane][16 B], so every fragment read is a conflict-free
// 16-byte read.  Chunks stream through a two-slot ring (one __shared__ array per slot, declared
// by the kernel) with double-buffered fragments; the LDS reads and the loads of later chunks
// are interleaved between the matrix-core instructions.
#pragma once
#include <hip/hip_runtime.h>

#include "ring.h"

namespace lrs {

typedef __attribute__((__vector_size__(4 * sizeof(double)))) double cg_f64x4;

constexpr int CG_BM = 64, CG_BN = 128, CG_KC = 16;   // workgroup tile, k per chunk
constexpr int CG_WN = 2;                             // waves: 2 (rows) x 2 (columns)
constexpr int CG_MB = 2, CG_NB = 4;                  // 16 x 16 accumulator blocks per wave
constexpr int CG_AT = CG_BM / 16, CG_BT = CG_BN / 16;
constexpr int CG_STAGE = (CG_AT + CG_BT) * 4096;     // LDS bytes of one chunk
constexpr int CG_LPW = CG_AT + CG_BT;                // loads per wave per chunk

// One workgroup tile: nch chunks of 16 k.  Wave w loads plane w / 2 (0 real, 1 imaginary),
// half w % 2 of every 16-row tile of a chunk; asrc[t] / bsrc[t] are the lane's sources for
// chunk 0 of A tile t (rows 16 t + l%16 of the tile) and B tile t, that is the plane's row
// start + 4 (l/16) + 2 (w%2); chunk c reads 16 c elements further.  cr, ci (wave (wm, wn),
// block (i, j); element e of a lane is row 4 e + lane/16, column lane%16 of the block) must
// be zero on entry (or hold what the tile adds to).
__device__ __forceinline__ void cgemm64_tile(const double* (&asrc)[CG_AT],
                                             const double* (&bsrc)[CG_BT], int nch, int wave,
                                             int lane, unsigned char* slot0,
                                             unsigned char* slot1, cg_f64x4 (&cr)[CG_MB][CG_NB],
                                             cg_f64x4 (&ci)[CG_MB][CG_NB]) {
  const int wm = wave / CG_WN, wn = wave % CG_WN;
  const int dofs = (wave >> 1) * 2048 + (wave & 1) * 1024;
  auto issue = [&](int c, unsigned char* dst) {
#pragma unroll
    for (int t = 0; t < CG_AT; ++t)
      __builtin_amdgcn_global_load_lds(
          (const void __attribute__((address_space(1)))*)(asrc[t] + c * CG_KC),
          (void __attribute__((address_space(3)))*)(dst + t * 4096 + dofs), 16, 0, 0);
#pragma unroll
    for (int t = 0; t < CG_BT; ++t)
      __builtin_amdgcn_global_load_lds(
          (const void __attribute__((address_space(1)))*)(bsrc[t] + c * CG_KC),
          (void __attribute__((address_space(3)))*)(dst + (CG_AT + t) * 4096 + dofs), 16, 0, 0);
  };
  // fragments of one chunk: value s of a lane is k = 4 (lane/16) + s
  struct Frag {
    cg_f64x4 ar[CG_MB], ai[CG_MB], br[CG_NB], bi[CG_NB];
  };
  auto load = [&](const unsigned char* sl, Frag& f) {
#pragma unroll
    for (int i = 0; i < CG_MB; ++i) {
      const unsigned char* t = sl + (wm * CG_MB + i) * 4096 + lane * 16;
      const double2 r0 = *(const double2*)(t), r1 = *(const double2*)(t + 1024);
      const double2 i0 = *(const double2*)(t + 2048), i1 = *(const double2*)(t + 3072);
      f.ar[i] = cg_f64x4{r0.x, r0.y, r1.x, r1.y};
      f.ai[i] = cg_f64x4{i0.x, i0.y, i1.x, i1.y};
    }
#pragma unroll
    for (int j = 0; j < CG_NB; ++j) {
      const unsigned char* t = sl + (CG_AT + wn * CG_NB + j) * 4096 + lane * 16;
      const double2 r0 = *(const double2*)(t), r1 = *(const double2*)(t + 1024);
      const double2 i0 = *(const double2*)(t + 2048), i1 = *(const double2*)(t + 3072);
      f.br[j] = cg_f64x4{r0.x, r0.y, r1.x, r1.y};
      f.bi[j] = cg_f64x4{i0.x, i0.y, i1.x, i1.y};
    }
  };
  auto mma = [&](const Frag& f) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < CG_MB; ++i)
#pragma unroll
        for (int j = 0; j < CG_NB; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.ar[i][s], f.br[j][s], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.ar[i][s], f.bi[j][s], ci[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-f.ai[i][s], f.bi[j][s], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.ai[i][s], f.br[j][s], ci[i][j], 0, 0, 0);
        }
  };
  // Chunk c sits in slot c % 2 with its fragments in register set c % 2.  Per step: barrier
  // (chunk c+1 landed, chunk c's slot read out), read chunk c+1's fragments, load chunk c+2
  // into chunk c's slot, matrix-core instructions of chunk c, with the reads and loads
  // interleaved between them.  Loads past the last chunk repeat it, so every step is one
  // basic block; an odd chunk count ends with the last chunk's instructions alone.
  constexpr int kMFMA = 0x008, kVMEM = 0x010, kDSREAD = 0x100;
  constexpr int NMF = 16 * CG_MB * CG_NB, NDS = 4 * (CG_MB + CG_NB), NVM = CG_LPW;
  constexpr int R = (NMF - NDS) / (NVM + 1), REST = NMF - NDS - R * NVM;
  auto sched = [] {
    sched_pairs<NDS, kMFMA, 1, kDSREAD, 1>();
    sched_pairs<NVM, kMFMA, R, kVMEM, 1>();
    __builtin_amdgcn_sched_group_barrier(kMFMA, REST, 0);
  };
  Frag fa, fb;
  issue(0, slot0);
  issue(min(1, nch - 1), slot1);
  ring_barrier<0>();
  load(slot0, fa);
  int c = 0;
  for (; c + 2 <= nch; c += 2) {
    ring_barrier<0>();
    load(slot1, fb);
    issue(min(c + 2, nch - 1), slot0);
    mma(fa);
    sched();
    ring_barrier<0>();
    load(slot0, fa);
    issue(min(c + 3, nch - 1), slot1);
    mma(fb);
    sched();
  }
  if (c < nch) mma(fa);
  ring_barrier<0>();
}

}  // namespace lrs
