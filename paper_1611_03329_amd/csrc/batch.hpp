// batch.hpp -- the step kernel over a table of lattices.
//
// Every lattice is stepped through a member table: a single lattice is a table
// of one; a batch's members share the lattice type, the storage precision and
// the time parity (a lattice whose parity differs takes one step of its own
// before it joins), so one launch of k_step advances all of them by one step:
// tile t belongs to the member whose tile range holds t, and is processed by
// the per-block body step_block on that member's state.  One kernel for both
// makes a member's trajectory bit for bit the same alone and in any batch.  The
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
  // the lattice's step count, one slot per parity: a step at parity p reads
  // clk[p] and writes clk[p ^ 1] = clk[p] + 1, so no launch reads what it writes
  uint32_t* clk;
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

// One time step of every member of a table: the step kernel of every lattice
// (a single lattice is a table of one member).  Tile t (blockDim.x nodes of one
// member) is taken by one block.  With nxcd > 1 the tile list is cut into nxcd
// contiguous ranges and block b (which the hardware places on XCD b % nxcd)
// walks range b % nxcd, so neighbouring tiles share an L2 cache; otherwise
// block b takes tiles b, b + gridDim.x, ...  A grid smaller than the tile count
// keeps its blocks resident and lets them walk several tiles (a persistent
// launch).  With nxcd > 1 the grid is a multiple of nxcd.
template <class Lat, class S, class C, bool ODD, int MODE, bool GEN, bool SEP>
__device__ __forceinline__ void step_tiles(const Member<S, C>* __restrict__ mem, int nmem, int ntiles, int nxcd) {
  int t, end, stride;
  if (nxcd > 1) {
    const int per = (ntiles + nxcd - 1) / nxcd;
    const int x = (int)blockIdx.x % nxcd;
    t = x * per + (int)blockIdx.x / nxcd;
    end = min(ntiles, (x + 1) * per);
    stride = (int)gridDim.x / nxcd;
  } else {
    t = (int)blockIdx.x;
    end = ntiles;
    stride = (int)gridDim.x;
  }
  for (; t < end; t += stride) {
    // odd steps walk the tiles backwards: they start on the tiles the even
    // step wrote last, which the last-level cache still holds
    const int tt = ODD ? ntiles - 1 - t : t;
    const int m = member_of(mem, nmem, tt);
    // the parameters are read in place: the general wall rules index their
    // per-face arrays with a per-node face number, which a private copy would
    // have to keep in scratch memory
    const KParams<C>& kp = mem[m].kp;
    const S sto = mem[m].sto;
    C* const snap = mem[m].snap;
    double* const part = mem[m].part;
    const int lb = tt - mem[m].block0;
    uint32_t* const clk = mem[m].clk;
    const uint32_t now = clk[ODD ? 1 : 0];
    const uint32_t seed = kStochastic<S> ? mix32(now) : 0u;
    if (lb == 0 && threadIdx.x == 0) gbl(clk)[ODD ? 0 : 1] = now + 1u;
    if constexpr (MODE == kModeCompare) {
      // a member that joined after the last snapshot has nothing to compare yet
      if (mem[m].check) step_block<Lat, S, C, ODD, kModeCompare, GEN, SEP>(kp, sto, snap, part, lb, seed);
      else step_block<Lat, S, C, ODD, kModePlain, GEN, SEP>(kp, sto, snap, part, lb, seed);
      // the block reduction's shared slots are reused by the next tile
      __syncthreads();
    } else if constexpr (MODE == kModeSpan) {
      // without a snapshot yet the member only takes one
      if (mem[m].check) step_block<Lat, S, C, ODD, kModeSpan, GEN, SEP>(kp, sto, snap, part, lb, seed);
      else step_block<Lat, S, C, ODD, kModeSnapshot, GEN, SEP>(kp, sto, snap, part, lb, seed);
      __syncthreads();
    } else {
      step_block<Lat, S, C, ODD, MODE, GEN, SEP>(kp, sto, snap, part, lb, seed);
    }
  }
}

// SEP (separable tiles: the link indices of the odd step from per-axis deltas)
// is compiled for FP16 storage only: there it takes 6-7 % of the odd step's
// vector instructions away and 7 % of its time.  With FP32 storage the
// registers the deltas occupy made the step slower.  It is a kernel of its
// own, not a branch: both address paths in one kernel exceed the register
// budget below.
//
// The step kernel with FP32 arithmetic (FP32 and FP16 storage) is held to 128
// registers, 4 wavefronts per SIMD: the general wall rules alone would need up
// to 157 and, sharing the kernel with the lean rules, cut every wavefront's
// occupancy to 3 (the channel ran 12-18 % slower).  With FP64 arithmetic the
// same limit would spill heavily, so that kernel keeps its own budget.
template <class Lat, class S, class C, bool ODD, int MODE, bool GEN, bool SEP>
__global__ void __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_step(const Member<S, C>* __restrict__ mem, int nmem, int ntiles, int nxcd) {
  step_tiles<Lat, S, C, ODD, MODE, GEN, SEP>(mem, nmem, ntiles, nxcd);
}
template <class Lat, class S, class C, bool ODD, int MODE, bool GEN>
__global__ void __launch_bounds__(kMaxBlock) k_step_fp64(const Member<S, C>* __restrict__ mem, int nmem,
                                                         int ntiles, int nxcd) {
  step_tiles<Lat, S, C, ODD, MODE, GEN, false>(mem, nmem, ntiles, nxcd);
}

// The step kernel for arithmetic type C (SEP: FP16 storage, odd step only).
template <class Lat, class S, class C, bool ODD, int MODE, bool GEN, bool SEP = false>
constexpr auto step_kernel() {
  static_assert(!SEP || (kStochastic<S> && ODD), "separable-tile indices are built for the FP16 odd step only");
  if constexpr (std::is_same<C, double>::value) return &k_step_fp64<Lat, S, C, ODD, MODE, GEN>;
  else return &k_step<Lat, S, C, ODD, MODE, GEN, SEP>;
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
