// rbdi_batch.hpp -- many independent instances (uneven grid sizes, same
// system and precision) advanced together: every phase of a step (seeding,
// each sweep of each RK stage) is ONE launch over a merged work list of all
// instances' tiles. The grid is persistent: a fixed number of blocks (or one
// block per item) walks the list, optionally with XCD-aware ranges so that
// the blocks of one XCD (blocks are dispatched round-robin over the 8 XCDs)
// work on a contiguous run of tiles. Phase boundaries stay kernel
// boundaries: a sweep reads what the previous sweep wrote anywhere in the
// instance, across XCDs, whose L2 caches are not coherent with each other.
//
// The per-cell arithmetic is the single-instance arithmetic (the same
// device bodies), so results do not depend on the tile shape, the block
// size, the grid or the batch composition.
#pragma once

#include "rbdi_kernels.hpp"

namespace rbdi {

template <typename T>
struct BatchInst {
  Params P;
  T* U[3];
  T* D;
  DevScalars* sc;
  double* cflpart;
  const SeedTask* tasks;
  int ntask;  // seeding tasks of the (static) band
  int par0;   // parity of the instance's next step when the batch was made
};

// One tile of one instance: local block coordinates and the local linear
// block index (CFL partial slots of the x sweep). For seeding, bx is the
// first task of a chunk of 256.
struct BatchItem {
  int inst, bx, by, bz;
  long long blin;
  int pad[2];
};

struct BatchArgs {
  int flip;              // steps taken by the batch (parity flips)
  double cfl, t_end;
  const double* dtfix;   // per instance: > 0 fixed dt, <= 0 CFL; null: CFL for all
  int in, out;           // state buffer indices of the stage
  int stage;
  double bcoef;
  int rhs_only;
  int nitems;
  int xcd;               // 1: XCD-aware item ranges
};

template <typename T>
__device__ inline StepArgs batch_step_args(const BatchInst<T>& bi, const BatchArgs& B, int inst) {
  StepArgs A{};
  A.par = bi.par0 ^ (B.flip & 1);
  A.cfl = B.cfl;
  A.t_end = B.t_end;
  A.dt_fixed = B.dtfix ? B.dtfix[inst] : 0.0;
  A.rhs_only = B.rhs_only;
  return A;
}

// Items of this block: [first, end) with the given stride.
__device__ inline void batch_items(const BatchArgs& B, int& first, int& end, int& stride) {
  const int g = (int)gridDim.x;
  if (B.xcd && g >= 8 && (g & 7) == 0) {
    const int per = g >> 3, x = (int)blockIdx.x & 7, slot = (int)blockIdx.x >> 3;
    const int chunk = (B.nitems + 7) >> 3;
    first = x * chunk + slot;
    end = min(B.nitems, (x + 1) * chunk);
    stride = per;
  } else {
    first = (int)blockIdx.x;
    end = B.nitems;
    stride = g;
  }
}

template <class S, typename T>
__global__ __launch_bounds__(256) void kb_sweep_x(const BatchInst<T>* __restrict__ I,
                                                 const BatchItem* __restrict__ items, BatchArgs B) {
  const int wpb = blockDim.x / kWave;
  int w, end, stride;
  batch_items(B, w, end, stride);
  for (; w < end; w += stride) {
    const BatchItem it = items[w];
    const BatchInst<T>& bi = I[it.inst];
    const StepArgs A = batch_step_args(bi, B, it.inst);
    const int nseg = (bi.P.n[0] + kOut - 1) / kOut;
    const int nparts = (nseg + wpb - 1) / wpb * wpb * bi.P.n[1] * bi.P.n[2];
    sweep_x_body<S, T>(bi.P, bi.U[B.in], bi.U[0], bi.D, nullptr, bi.U[B.out], bi.sc, bi.cflpart, A, B.bcoef, B.stage,
                       it.bx, it.by, it.bz, it.blin, wpb, nparts);
  }
}

// Tile of tc columns in dynamic LDS (S::NF * tc * kRS values).
template <class S, typename T, int DIR, int MODE, bool REDUCE>
__global__ __launch_bounds__(kTileThreads) void kb_sweep_tile(const BatchInst<T>* __restrict__ I,
                                                    const BatchItem* __restrict__ items, BatchArgs B, int tc) {
  extern __shared__ double lds_dyn[];
  T* tile = reinterpret_cast<T*>(lds_dyn);
  int w, end, stride;
  batch_items(B, w, end, stride);
  for (; w < end; w += stride) {
    __syncthreads();  // the previous item's tile has been stored
    const BatchItem it = items[w];
    const BatchInst<T>& bi = I[it.inst];
    const StepArgs A = batch_step_args(bi, B, it.inst);
    sweep_tile_body<S, T, DIR, MODE, REDUCE>(bi.P, bi.U[B.in], bi.D, bi.sc, bi.cflpart, A, it.bx, it.by, it.bz,
                                             tile, tc);
  }
}

template <class S, typename T>
__global__ __launch_bounds__(256) void kb_seed(const BatchInst<T>* __restrict__ I,
                                              const BatchItem* __restrict__ items, BatchArgs B) {
  int w, end, stride;
  batch_items(B, w, end, stride);
  for (; w < end; w += stride) {
    const BatchItem it = items[w];
    const BatchInst<T>& bi = I[it.inst];
    const StepArgs A = batch_step_args(bi, B, it.inst);
    if (step_done(bi.sc, A)) continue;  // uniform over the block
    const int b = it.bx + (int)threadIdx.x;
    const double tc = bi.sc->t[A.par] - bi.sc->t_motion;
    int n = 0;
    if (b < bi.ntask) {
      seed_one<S, T>(bi.P, bi.U[0], bi.tasks[b], tc);
      n = 1;
    }
    wave_count_add(&bi.sc->seeded, n);
  }
}

}  // namespace rbdi
