// Per-lane index maps of the continuous-Galerkin cell kernel, shared by the
// kernel (kernels.hip) and the host-side check of every operator set-up
// (tetmf.cpp).  Each function states which row of a per-cell array, or which
// entry of an LDS table, one lane reads; the host check enumerates every
// lane of the kernel instantiation an operator will launch and verifies that
// each read stays inside its array and that every 32-bit byte offset the
// kernel forms fits at the largest mesh the set-up accepts.  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace tetmf {
namespace lanes {

// Accumulator element r of lane group g of a 16x16x4 matrix-core product
// holds output row g + 4 r (FP64) or 4 g + r (FP32 and the BF16-operand
// engine, which uses the FP32 accumulator layout).
__host__ __device__ constexpr int acc_row(int esize, int g, int r) { return esize == 8 ? g + 4 * r : 4 * g + r; }

// DoFs integrated on the 16-row products, and those left to the tail
// (DoFs 16.., FP64: the 4x4x4 products, BF16: the second 16x16x32 chain).
__host__ __device__ constexpr int n_main(int ndof) { return ndof < 16 ? ndof : 16; }
__host__ __device__ constexpr int n_tail(int ndof) { return ndof - n_main(ndof); }

// Row of the [n_dof][ncp] slot-position array read for accumulator element r
// of lane group g, or -1: rows beyond the cell's DoFs (fewer than 16 at
// p <= 2) have no slot and are not read.  The kernel reads it from the row
// base acc_row(0, r) with the lane part acc_row(g, 0) in its offset.
__host__ __device__ constexpr int pos_row(int esize, int ndof, int g, int r) {
  return acc_row(esize, g, r) < n_main(ndof) ? acc_row(esize, g, r) : -1;
}
// Row read for the tail DoF of lane group g (lane groups g >= n_tail repeat
// the last tail row and write nothing), or -1 without a tail.
__host__ __device__ constexpr int pos_tail_row(int ndof, int g) {
  return n_tail(ndof) > 0 ? 16 + (g < n_tail(ndof) - 1 ? g : n_tail(ndof) - 1) : -1;
}

// Library layout of per-point cell data (coefficients, their gradients,
// source samples): 16-cell tiles of consecutive library cells, each tile
// holding its n_q points one after another with 16 values (one per cell)
// per point, [ceil(n_cell / 16)][n_q][16].  A tile's data is one contiguous
// run of 16 n_q values; the last tile is padded.
__host__ __device__ constexpr long cell_data_index(int nq, int q, long cell) {
  return ((cell >> 4) * nq + q) * 16 + (cell & 15);
}
__host__ __device__ constexpr long cell_data_size(int nq, long ncell) { return (long)nq * ((ncell + 15) / 16 * 16); }

// Per-point geometry of curved cells (7 values per point: G and |det J|) in
// 16-cell tiles, [ncp / 16][7][n_q][16]: one tile's geometry is one
// contiguous run of 7 16 n_q values.
__host__ __device__ constexpr long curved_geo_index(int nq, int c, int q, long cell) {
  return (((cell >> 4) * 7 + c) * nq + q) * 16 + (cell & 15);
}

// Point of the lane's k-th group read from the per-point cell data, relative
// to the group base 4 k: lane group g in a full group of four points, clamped
// to the last point in a partly used last group (whose value is then masked).
__host__ __device__ constexpr int kappa_lane_row(int nq, int g, int k) {
  return 4 * k + 3 < nq ? g : (g + 4 * k < nq - 1 ? g + 4 * k : nq - 1) - 4 * k;
}

// Row of the block-local index array [n_dof][256] read for operand row j of
// an interpolation (rows beyond the cell's DoFs read the last valid row and
// are zeroed afterwards).
__host__ __device__ constexpr int operand_row(int ndof, int j) { return j < ndof ? j : ndof - 1; }

}  // namespace lanes
}  // namespace tetmf
