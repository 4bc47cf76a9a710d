// Internal declarations of the fkdmft library (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fk {

// Interleaved complex number, the element type of every device matrix.
template <typename T> struct alignas(2 * sizeof(T)) cplx { T re, im; };
typedef cplx<double> c64;
typedef cplx<float> c32;

// One matrix of a batched Gauss-Jordan inversion.  x + xoff is element (0,0)
// of an n x n row-major matrix with leading dimension ld (elements).
// piv + ioff and rowcol + ioff hold n ints each: piv[c] = row chosen as pivot
// for column c, rowcol[r] = column whose pivot row is r (-1 while unpivoted).
// bbuf + boff holds kBRows rows of ld elements: the gathered pivot rows of the
// one or two outer blocks whose transforms the next update applies.
struct MatDesc {
  long long xoff;
  long long boff;
  int n;
  int ld;
  int ioff;
  int status_idx;
};

// Tile of an update launch: (matrix, row tile, column tile) and the transform
// it applies: C <- mask(C) + M B with M the kw columns starting at column
// jb * kNBO (the transformed identity columns of one or two outer blocks),
// B the rows b0 .. b0 + kw of the side buffer, and the rows whose pivot column
// lies in [jb kNBO, jb kNBO + kw) masked.  Items of one launch may carry
// different transforms (uneven batches: each matrix follows its own schedule).
struct TileItem {
  int mat;
  short tr;
  short tc;
  short jb;
  short kw;
  short b0;
  short pad;
};

#ifndef FK_GROUP_BLOCKS
#define FK_GROUP_BLOCKS 4
#endif
constexpr int kNB = 64;          // inner panel width (columns)
constexpr int kNBO = 128;        // outer block: two inner panels
constexpr int kGroup = FK_GROUP_BLOCKS;  // outer blocks per delayed trailing update
constexpr int kBRows = kGroup * kNBO;    // side buffer rows: one group's pivot rows
constexpr int kPhases = 3;       // update launches per outer step (push_tiles)
constexpr int kTile = 64;        // trailing-update tile (rows = cols)
constexpr int kKC = 16;          // K chunk of the trailing update
constexpr int kIB = 8;           // panel columns eliminated in registers at once
constexpr int kPanelThreads = 512;
constexpr int kGemmThreads = 256;
constexpr int kMaxN = 5120;      // largest matrix the inversion supports

// Outer blocks are applied to the columns outside them in groups of up to
// kGroup blocks, counted from the last block ((L-g+1 .. L), (L-2g+1 .. L-g),
// ...; L = nouter - 1, g = kGroup); the first nouter mod g blocks form a
// shorter group.  A group's trailing update is delayed until all its blocks
// are factored and then applies their transforms at once (K up to kBRows):
// with M_i the transformed identity columns of the group's blocks and B_i
// their gathered pivot rows (values before the group's first step outside
// the group),
//   C <- mask(C) + [M_1' | ... | M_g] [B_1; ...; B_g],
// where M_i' is M_i brought up to date by the transforms of the later blocks
// of the group (each block, once factored, updates the earlier blocks'
// columns: M <- mask(M) + M_p B_p), which equals the steps one after the
// other.  Before block p of a group is factored its own columns receive the
// transforms of the group's blocks before it in the same form.
// Position of block S of an n-row matrix within its group (0 = first).
__host__ __device__ inline int block_pos(int n, int S) {
  const int r = ((n + kNBO - 1) / kNBO) % kGroup;
  return S < r ? S : (S - r) % kGroup;
}
// Whether block S is the last of its group (its step runs the trailing update).
__host__ __device__ inline bool block_last(int n, int S) {
  const int nout = (n + kNBO - 1) / kNBO;
  const int r = nout % kGroup;
  return S + 1 == nout || (S < r ? S == r - 1 : (S - r) % kGroup == kGroup - 1);
}
// First side-buffer row of block S's gathered pivot rows.
__host__ __device__ inline int block_brow(int n, int S) {
  return block_pos(n, S) * kNBO;
}

// Outer step S of the blocked in-place Gauss-Jordan inversion, pieces:
//   panel   one workgroup per matrix factors the outer block [S*kNBO, +kNBO)
//   gather  copies the pivot rows of block S into the side buffer
//   fix     the block's columns of the rows pivoted before step S
//   update  C <- mask(C) + M B on the listed tiles (per-item transform)
template <typename T>
hipError_t gje_panel(cplx<T>* x, int* piv, int* rowcol, const MatDesc* d,
                     int nmat, int nmax, int S, int* status, hipStream_t st);
template <typename T>
hipError_t gje_gather(const cplx<T>* x, cplx<T>* bbuf, const int* piv,
                      const MatDesc* d, int nmat, int S, hipStream_t st);
template <typename T>
hipError_t gje_fix(cplx<T>* x, const cplx<T>* bbuf, const int* piv,
                   const MatDesc* d, int nmat, int S, hipStream_t st);
// variant 0: 64 x 64 tiles (256 threads); 1: 128 x 64 tiles (512 threads).
// TileItem.tr counts tiles of tile_rows(variant) rows.
template <typename T>
hipError_t gje_update(cplx<T>* x, const cplx<T>* bbuf, const int* rowcol,
                      const MatDesc* d, const TileItem* items, int nitems,
                      int variant, hipStream_t st);
inline int tile_rows(int variant) { return variant == 1 ? 128 : 64; }

}  // namespace fk
