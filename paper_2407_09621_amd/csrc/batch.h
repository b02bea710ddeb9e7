// Work lists passed by value in kernel arguments: up to kMaxBatch problems of
// the same degree per launch.  Each problem owns a contiguous range of work
// items (tiles, patches, coarse cells); a workgroup or wave finds its problem
// from the range starts, which are uniform kernel arguments.
#pragma once
#include <hip/hip_runtime.h>

namespace sipg {

constexpr int kMaxBatch = 16;

template <typename T>
struct Desc {
  const T* in;   // apply: u; patch: r; transfers: input; coarse: b
  T* out;        // apply: v; patch: x; transfers: output; coarse: x
  const T* aux;  // apply: b for the residual form, else unused
  T h;           // cell size of the level
  int n;         // cells per direction (transfers: coarse cells)
  int a0, a1, a2;  // apply: tx, ntx, blk; patch: npx, npy, npatch
};

template <typename T>
struct Batch {
  int count;
  int start[kMaxBatch + 1];  // work-item range of problem p: [start[p], start[p+1])
  Desc<T> d[kMaxBatch];
};

template <typename T>
__device__ __forceinline__ int batch_find(const Batch<T>& B, int item) {
  int p = 0;
  while (p + 1 < B.count && item >= B.start[p + 1]) ++p;
  return p;
}

// host-side job descriptions
struct ApplyJob {
  const void* u;
  void* v;
  const void* b;  // nullptr: v = A u; else v = b - A u
  int n;
  double h;
  int order = 0;  // tile order block (divides n); 0 = default (8 if it divides n, else 1)
};
struct PatchJob {
  const void* r;
  void* x;
  int n;
  double h;
  const void* b = nullptr;  // set: fused colour step, r = x_in, x = x_out, b = right-hand side
};
struct TransferJob {
  const void* in;
  void* out;
  int nc;  // coarse cells per direction
};
struct CoarseJob {
  const void* b;
  void* x;
  int n0;
  double h;
};

}  // namespace sipg
