// One launch path for every kernel of the factorization, single or batched.
//
// Each kernel is a template whose last parameter B selects where its
// parameter struct comes from: B = false takes it by value (one problem);
// B = true reads entry blockIdx.z of a device array (one entry per problem of
// a batch) and returns at once for blocks past that problem's own grid
// (every parameter struct carries its grid extents gx, gy).
//
// launch_k() launches the single form directly, or, while a Recorder is
// installed on the calling thread, appends {batched kernel, grid, block,
// parameters} to it instead.  The batch planner runs the ordinary
// single-problem orchestration once per problem under a recorder and turns
// the records into grouped launches.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <vector>

namespace pbq {

struct LaunchRec {
  const void* fn = nullptr;  // batched form of the kernel
  dim3 grid, block;
  std::vector<unsigned char> params;
};

struct Recorder {
  std::vector<LaunchRec> recs;
};

// Recorder of the calling thread (nullptr: launch directly).
Recorder*& current_recorder();

#define PBQ_GRID unsigned gx = 1, gy = 1

// Parameters of kernel instance B: by value, or entry blockIdx.z of the batch
// array.  `past` tells a batched block that it lies outside its problem's grid.
template <bool B, class P>
__device__ __forceinline__ P kparams(const P* pb, const P& ps, bool& past) {
  if constexpr (B) {
    const P p = pb[blockIdx.z];
    past = blockIdx.x >= p.gx || blockIdx.y >= p.gy;
    return p;
  } else {
    past = false;
    return ps;
  }
}

template <class P>
hipError_t launch_k(void (*k_single)(const P*, P), void (*k_batched)(const P*, P), dim3 grid,
                    dim3 block, hipStream_t s, P p) {
  p.gx = grid.x;
  p.gy = grid.y;
  if (Recorder* r = current_recorder()) {
    LaunchRec rec;
    rec.fn = (const void*)k_batched;
    rec.grid = grid;
    rec.block = block;
    rec.params.assign((const unsigned char*)&p, (const unsigned char*)&p + sizeof(P));
    r->recs.push_back(std::move(rec));
    return hipSuccess;
  }
  hipLaunchKernelGGL(k_single, grid, block, 0, s, (const P*)nullptr, p);
  return hipGetLastError();
}

}  // namespace pbq
