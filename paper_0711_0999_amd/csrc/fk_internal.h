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

constexpr int kNB = 64;          // inner panel width (columns)
constexpr int kNBO = 128;        // outer block: two inner panels
constexpr int kBRows = 2 * kNBO; // side buffer rows: two outer blocks' pivot rows
constexpr int kPhases = 3;       // update launches per outer step (push_tiles)
constexpr int kTile = 64;        // trailing-update tile (rows = cols)
constexpr int kKC = 16;          // K chunk of the trailing update
constexpr int kIB = 8;           // panel columns eliminated in registers at once
constexpr int kPanelThreads = 512;
constexpr int kGemmThreads = 256;
constexpr int kMaxN = 5120;      // largest matrix the inversion supports

// Outer blocks are applied to the columns outside them one or two at a time.
// Counted from the last block, blocks pair up ((L-1, L), (L-3, L-2), ...; L =
// nouter - 1); with an odd count block 0 stays single.  A pair's trailing
// update is delayed until both blocks are factored and then applies the two
// transforms at once (K up to 2 kNBO): with M1, M2 the transformed identity
// columns and B1, B2 the gathered pivot rows of the two blocks,
//   C <- mask(C) + [M1' | M2] [B1; B2],  M1' = mask(M1) + M2 B2[:, block 1],
// which equals the two steps one after the other.  Role of block S of an
// n-row matrix: 0 single, 1 first of a pair, 2 second of a pair.
__host__ __device__ inline int block_role(int n, int S) {
  const int nout = (n + kNBO - 1) / kNBO;
  if ((nout & 1) && S == 0) return 0;
  return ((nout - 1 - S) & 1) == 0 ? 2 : 1;
}
// First side-buffer row of block S's gathered pivot rows.
__host__ __device__ inline int block_brow(int n, int S) {
  return block_role(n, S) == 2 ? kNBO : 0;
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
