// Workgroup -> tile numbering for the 8-XCD MI355X.
//
// The dispatcher hands the workgroups of a launch to the 8 XCDs round-robin
// (workgroup b runs on XCD b mod 8), and each XCD has its own L2.  Element
// kernels renumber their workgroups so that every XCD receives one
// contiguous range of logical ids.  Elements are numbered x-fastest, so a
// contiguous range of elements is a slab of the mesh, and the face data a
// workgroup reads from its neighbours were mostly fetched into the same L2
// by a workgroup of the same XCD.  Every kernel uses the same numbering, so
// an element stays on one XCD from kernel to kernel.
#pragma once
#include <hip/hip_runtime.h>

namespace sisdc {

constexpr int kXcd = 8;

// Logical id of workgroup b in a grid of G workgroups (a bijection of
// [0, G)): XCD x receives ids [x*(G/8) + min(x, G%8), ...) in dispatch order.
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int x = b % kXcd, j = b / kXcd, per = G / kXcd, rem = G % kXcd;
  return x * per + (x < rem ? x : rem) + j;
}

// The contiguous range [t0, t1) of the nt tiles that this workgroup visits
// when a grid of gridDim.x <= nt workgroups loops over the tiles.
__device__ __forceinline__ void tile_range(int nt, int& t0, int& t1) {
  const long lb = xcd_block(blockIdx.x, gridDim.x);
  t0 = (int)(lb * nt / gridDim.x);
  t1 = (int)((lb + 1) * nt / gridDim.x);
}

}  // namespace sisdc
