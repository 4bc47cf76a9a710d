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
// bbuf + boff holds kNBO rows of ld elements: the gathered old pivot rows of
// the current outer step.
struct MatDesc {
  long long xoff;
  long long boff;
  int n;
  int ld;
  int ioff;
  int status_idx;
};

// Tile of the trailing update: (matrix, row tile, column tile) of kTile.
struct TileItem {
  int mat;
  short tr;
  short tc;
};

constexpr int kNB = 64;          // inner panel width (columns)
constexpr int kNBO = 128;        // outer block: two inner panels
constexpr int kTile = 64;        // trailing-update tile (rows = cols)
constexpr int kKC = 16;          // K chunk of the trailing update
constexpr int kIB = 8;           // panel columns eliminated in registers at once
constexpr int kPanelThreads = 512;
constexpr int kGemmThreads = 256;
constexpr int kMaxN = 5120;      // largest matrix the inversion supports

// Outer step S of the blocked in-place Gauss-Jordan inversion, pieces:
//   panel   one workgroup per matrix factors the outer block [S*kNBO, +kNBO)
//   gather  copies the old pivot rows of outer step S into the side buffer
//   fix     the block's columns of the rows pivoted before step S
//   update  C <- mask(C) + M B on the listed tiles (K = outer block width)
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
                      int S, int variant, hipStream_t st);
inline int tile_rows(int variant) { return variant == 1 ? 128 : 64; }

}  // namespace fk
