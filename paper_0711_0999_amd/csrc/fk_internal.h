// Internal declarations of the fkdmft library (HIP, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fk {

// Interleaved complex number, the element type of every device matrix.
template <typename T> struct alignas(2 * sizeof(T)) cplx { T re, im; };
typedef cplx<double> c64;
typedef cplx<float> c32;

// One matrix of a batched Gauss-Jordan inversion.  x points at element (0,0)
// of an n x n row-major matrix with leading dimension ld (elements); piv and
// rowcol point at n ints each: piv[c] = row chosen as pivot for column c,
// rowcol[r] = column whose pivot row is r (-1 while r is unpivoted).
struct MatDesc {
  long long xoff;   // element offset of the matrix in the batch buffer
  int n;
  int ld;
  int ioff;         // int offset of piv / rowcol for this matrix
  int status_idx;   // slot in the status array
};

// Work item of one inversion step: (matrix, column stripe).
struct WorkItem {
  int mat;
  int stripe;
};

constexpr int kNB = 64;        // panel width = stripe width (columns)
constexpr int kTM = 64;        // row tile of the trailing update
constexpr int kIB = 4;         // inner panel block held in registers
constexpr int kThreads = 256;  // workgroup size of the step kernel
constexpr int kMaxN = 2304;    // largest matrix the step kernel supports

// Launch one step of the blocked in-place Gauss-Jordan inversion for a batch.
// step = -1 factors the first panel only.  items[0..nitems) on the device.
template <typename T>
hipError_t gje_step(cplx<T>* xbuf, int* pivbuf, int* rowcolbuf,
                    const MatDesc* descs, const WorkItem* items, int nitems,
                    int step, int* status, int grid, hipStream_t st);

// Dynamic LDS bytes used by gje_step for element type T.
template <typename T> size_t gje_lds_bytes();

}  // namespace fk
