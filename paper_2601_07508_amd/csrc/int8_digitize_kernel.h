// Digit planes of the INT8-digit form: entries of A and B written as D
// signed base-256 digits, one int8 plane per digit (the digit GEMM in
// int8_digits_kernel.h reads them).  A plane of R rows by kp k-bytes is
// stored in 1 KB blocks of 16 rows by 64 k-bytes (plane_at), R rounded up to
// 16: the GEMM's copies then read 1 KB contiguous runs, and a row group's
// successive k-stages follow one another in memory.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mmp {
namespace i8d {

// byte offset of (row r, k-byte c) within a plane of kp k-bytes per row
__device__ __forceinline__ int64_t plane_at(int64_t r, int64_t c, int64_t kp) {
  return (r >> 4) * (kp << 4) + (c >> 6) * 1024 + (r & 15) * 64 + (c & 63);
}
// bytes of one plane of `rows` rows
__device__ __forceinline__ int64_t plane_size(int64_t rows, int64_t kp) { return ((rows + 15) & ~(int64_t)15) * kp; }

// Signed base-256 digits of an integer v with -128 R <= v <= 127 R,
// R = (256^D - 1) / 255: the low byte read as int8 is the digit, and the
// exact quotient (v - d) / 256 carries on.
template <int D>
__device__ __forceinline__ void digits_of_int(int64_t v, int8_t (&d)[D]) {
#pragma unroll
  for (int i = 0; i < D; i++) {
    const int8_t di = (int8_t)(v & 0xff);
    d[i] = di;
    v = (v - di) >> 8;
  }
}

// Entry loaders.  Residues: x in [0, p) stored as binary64; the digits are
// those of x' = x, or x - p when x exceeds 127 R (then x' >= -128 R because
// p <= 256^D).  Integers: uint64 entries below 2^62, taken as they are.
struct ResidueIn {
  const double* X;
  int64_t p, top;
  // x < 2^52 is an integer: x + 2^52 is exact and its significand is x
  __device__ __forceinline__ int64_t conv(double x) const {
    const int64_t v = __double_as_longlong(x + 4503599627370496.0) - 0x4330000000000000ll;
    return v > top ? v - p : v;
  }
  __device__ __forceinline__ int64_t operator()(int64_t idx) const { return conv(X[idx]); }
  // 8 entries from a 16-byte aligned address
  __device__ __forceinline__ void load8(int64_t idx, int64_t (&v)[8]) const {
    const double2* q = (const double2*)(X + idx);
#pragma unroll
    for (int h = 0; h < 4; h++) {
      const double2 w = q[h];
      v[2 * h] = conv(w.x);
      v[2 * h + 1] = conv(w.y);
    }
  }
};
struct IntegerIn {
  const uint64_t* X;
  __device__ __forceinline__ int64_t operator()(int64_t idx) const { return (int64_t)X[idx]; }
  __device__ __forceinline__ void load8(int64_t idx, int64_t (&v)[8]) const {
    const ulonglong2* q = (const ulonglong2*)(X + idx);
#pragma unroll
    for (int h = 0; h < 4; h++) {
      const ulonglong2 w = q[h];
      v[2 * h] = (int64_t)w.x;
      v[2 * h + 1] = (int64_t)w.y;
    }
  }
};

// A (rows x cols, row-major, ld) -> D planes of rows x kp, k zero-padded to kp.
// A workgroup covers 16 rows by 128 columns, two whole 1 KB blocks of every
// plane: grid x over 128-column chunks, y over 16-row groups (strided).  Each
// thread digitises 8 consecutive columns of one row (16 threads read 1 KB of
// a row) and stores one 8-byte word per plane.  VEC: the row's entries are
// 16-byte aligned (aligned base, even ld), so whole groups of 8 load as four
// 16-byte vectors.
// One workgroup's part: column chunk bx, row groups by, by + gy, ...
template <int D, class In, bool VEC>
__device__ __forceinline__ void digitize_rows_part(const In& X, int64_t rows, int64_t cols, int64_t ld, int64_t kp,
                                                   int8_t* __restrict__ out, int64_t bx, int64_t by, int64_t gy) {
  const int64_t c0 = bx * 128 + (threadIdx.x & 15) * 8;
  if (c0 >= kp) return;
  const int64_t plane = plane_size(rows, kp);
  for (int64_t r = by * 16 + (threadIdx.x >> 4); r < rows; r += gy * 16) {
    int64_t v[8];
    if (VEC && c0 + 8 <= cols) {
      X.load8(r * ld + c0, v);
    } else {
#pragma unroll
      for (int e = 0; e < 8; e++) v[e] = (c0 + e < cols) ? X(r * ld + c0 + e) : 0;
    }
    uint64_t packed[D];
#pragma unroll
    for (int i = 0; i < D; i++) packed[i] = 0;
#pragma unroll
    for (int e = 0; e < 8; e++) {
      int8_t d[D];
      digits_of_int<D>(v[e], d);
#pragma unroll
      for (int i = 0; i < D; i++) packed[i] |= (uint64_t)(uint8_t)d[i] << (8 * e);
    }
#pragma unroll
    for (int i = 0; i < D; i++) *(uint64_t*)(out + i * plane + plane_at(r, c0, kp)) = packed[i];
  }
}

template <int D, class In, bool VEC>
__global__ __launch_bounds__(256) void digitize_rows_kernel(In X, int64_t rows, int64_t cols, int64_t ld,
                                                            int64_t kp, int8_t* __restrict__ out) {
  digitize_rows_part<D, In, VEC>(X, rows, cols, ld, kp, out, blockIdx.x, blockIdx.y, gridDim.y);
}

// B (krows x ncols, row-major, ld) -> D transposed planes of ncols x kp.
// 64 x 64 tiles through LDS so that both the reads (along n) and the writes
// (16 columns' 64 k-bytes, one whole block, per 256 threads) are contiguous.
// One workgroup's part: 64 x 64 tile number `t` (n fastest), through `tile`.
template <int D, class In>
__device__ __forceinline__ void digitize_cols_part(const In& X, int64_t krows, int64_t ncols, int64_t ld, int64_t kp,
                                                   int8_t* __restrict__ out, int64_t t,
                                                   uint8_t (&tile)[D][64][64 + 4]) {
  const int64_t tiles_n = (ncols + 63) / 64;
  const int64_t k0 = (t / tiles_n) * 64;
  const int64_t n0 = (t % tiles_n) * 64;
  const int tid = threadIdx.x;
  // read: 64 k-rows x 64 columns; thread tid takes column tid % 64 of k-rows
  // tid / 64 + 4 u, u < 16, all 16 loads issued before any is used
  const int nn = tid % 64, kb = tid / 64;
  const int64_t col = n0 + nn;
  int64_t v[16];
#pragma unroll
  for (int u = 0; u < 16; u++) {
    const int64_t row = k0 + kb + 4 * u;
    v[u] = (row < krows && col < ncols) ? X(row * ld + col) : 0;
  }
#pragma unroll
  for (int u = 0; u < 16; u++) {
    int8_t d[D];
    digits_of_int<D>(v[u], d);
#pragma unroll
    for (int i = 0; i < D; i++) tile[i][nn][kb + 4 * u] = (uint8_t)d[i];
  }
  __syncthreads();
  // write: for each plane and column, 64 k-bytes as 16 words
  const int64_t plane = plane_size(ncols, kp);
#pragma unroll
  for (int u = 0; u < 4 * D; u++) {  // D x 64 columns x 16 words over 256 threads
    const int e = tid + 256 * u;
    const int i = e / (64 * 16);
    const int rem = e % (64 * 16);
    const int cn = rem / 16, w = rem % 16;
    const int64_t ocol = n0 + cn, kq = k0 + 4 * w;
    if (ocol < ncols && kq < kp)  // 4 digit bytes, k-order, read as one word (rows are 68 bytes)
      *(uint32_t*)(out + i * plane + plane_at(ocol, kq, kp)) = *(const uint32_t*)&tile[i][cn][4 * w];
  }
}

template <int D, class In>
__global__ __launch_bounds__(256) void digitize_cols_kernel(In X, int64_t krows, int64_t ncols, int64_t ld,
                                                            int64_t kp, int8_t* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint8_t tile[D][64][64 + 4];
  digitize_cols_part<D, In>(X, krows, ncols, ld, kp, out, blockIdx.x, tile);
}

// A's rows and B's columns of one product in a single launch: workgroups
// below gx * gy take the row part (column chunk b % gx, row groups b / gx +
// gy i), the rest the 64 x 64 column tiles.  One kernel boundary fewer, and
// the two passes' tails overlap.
template <int D, class In, bool VEC>
__global__ __launch_bounds__(256) void digitize_pair_kernel(In XA, int64_t m, int64_t k, int64_t lda, In XB,
                                                            int64_t n, int64_t ldb, int64_t kp,
                                                            int8_t* __restrict__ outA, int8_t* __restrict__ outB,
                                                            int64_t gx, int64_t gy) {
  __shared__ __attribute__((aligned(16))) uint8_t tile[D][64][64 + 4];
  const int64_t b = blockIdx.x, nrows = gx * gy;
  if (b < nrows)  // uniform per workgroup: the row part has no barrier
    digitize_rows_part<D, In, VEC>(XA, m, k, lda, kp, outA, b % gx, b / gx, gy);
  else
    digitize_cols_part<D, In>(XB, k, n, ldb, kp, outB, b - nrows, tile);
}

}  // namespace i8d
}  // namespace mmp
