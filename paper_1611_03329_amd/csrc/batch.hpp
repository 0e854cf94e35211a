// batch.hpp -- many lattices advanced by one launch per time step.
//
// Members of a batch share the lattice type, the storage precision and the
// time parity (a lattice whose parity differs takes one step of its own before
// it joins), so one launch of k_step_batch advances all of them by one step:
// tile t belongs to the member whose tile range holds t, and is processed by
// the same per-block body as the single-lattice kernel on that member's state.  The
// residual check follows one schedule for the whole batch; per-member partials
// are folded by k_fold_members into each member's result area and into one
// batch-wide array that a single copy brings to the host.
#pragma once

#include "kernels.hpp"

namespace lbm {

template <class S, class C>
struct Member {
  KParams<C> kp;
  S sto;          // populations
  C* snap;        // residual snapshot, 4 planes of kp.n
  double* part;   // per-block partials (member-local block index)
  double* res;    // the member's own 8-double result area
  int block0;     // first tile of the member in the batch's tile list
  int nblocks;    // tiles of the member
  int check;      // the member's snapshot is valid: a compare step compares it
};

// Member owning block b: members are sorted by block0 and block0 of the first is 0.
template <class M>
__device__ __forceinline__ int member_of(const M* __restrict__ mem, int nmem, int b) {
  int lo = 0, hi = nmem - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (mem[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One time step of every member.  Tile t (blockDim.x nodes of one member) is
// taken by block t mod gridDim.x: with a grid smaller than the tile count the
// blocks stay resident and walk the tile list (a persistent launch).
template <class Lat, class S, class C, bool ODD, int MODE, bool GEN>
__global__ void __launch_bounds__(kMaxBlock) k_step_batch(const Member<S, C>* __restrict__ mem, int nmem,
                                                          int ntiles) {
  for (int t = (int)blockIdx.x; t < ntiles; t += (int)gridDim.x) {
    const int m = member_of(mem, nmem, t);
    // private copies, as the single-lattice kernel receives them: the step's
    // arithmetic then compiles exactly as there
    const KParams<C> kp = mem[m].kp;
    const S sto = mem[m].sto;
    C* const snap = mem[m].snap;
    double* const part = mem[m].part;
    const int lb = t - mem[m].block0;
    if constexpr (MODE == kModeCompare) {
      // a member that joined after the last snapshot has nothing to compare yet
      if (mem[m].check) step_block<Lat, S, C, ODD, kModeCompare, GEN>(kp, sto, snap, part, lb);
      else step_block<Lat, S, C, ODD, kModePlain, GEN>(kp, sto, snap, part, lb);
      // the block reduction's shared slots are reused by the next tile
      __syncthreads();
    } else if constexpr (MODE == kModeSpan) {
      // without a snapshot yet the member only takes one
      if (mem[m].check) step_block<Lat, S, C, ODD, kModeSpan, GEN>(kp, sto, snap, part, lb);
      else step_block<Lat, S, C, ODD, kModeSnapshot, GEN>(kp, sto, snap, part, lb);
      __syncthreads();
    } else {
      step_block<Lat, S, C, ODD, MODE, GEN>(kp, sto, snap, part, lb);
    }
  }
}

// Block m folds member m's partials of the last compare step and forms its
// residual (as k_fold_partials + k_residual_final do for one lattice); the
// result goes to the member's own area and to out[m * kPartStride ...].
template <class S, class C>
__global__ void __launch_bounds__(kMaxBlock) k_fold_members(const Member<S, C>* __restrict__ mem,
                                                            double* __restrict__ out) {
  const Member<S, C>& M = mem[blockIdx.x];
  if (!M.check) return;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < M.nblocks; b += blockDim.x) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] += M.part[(size_t)b * kPartStride + j];
    v[4] = pick_max(v[4], M.part[(size_t)b * kPartStride + 4]);
  }
  block_reduce<5>(v, 1u << 4);
  if (threadIdx.x == 0) {
    finish_residual(v, M.res);
#pragma unroll
    for (int j = 0; j < 8; ++j) out[(size_t)blockIdx.x * kPartStride + j] = M.res[j];
  }
}

}  // namespace lbm
