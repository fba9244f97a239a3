// Internal declarations shared by the host setup (tetmf.cpp) and the HIP
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tetmf {

// Cells handled by one workgroup pass of the continuous-Galerkin kernel.  The
// block's DoFs are staged in LDS; DoFs touched only by one block are written
// directly, the others go through per-block partial sums (see cg_reduce).
constexpr int kBlockCells = 256;
// Cells per MFMA tile (the N dimension of the 16x16 matrix-core products).
constexpr int kTile = 16;
constexpr int kWaves = 8;                  // waves per workgroup
constexpr int kThreads = kWaves * 64;      // threads per workgroup
constexpr int kTilesPerWave = kBlockCells / kTile / kWaves;

enum Mode { MODE_APPLY = 0, MODE_BACKWARD = 1, MODE_DIAG = 2, MODE_LOAD = 3 };
enum Prec { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

// Device-side description of a continuous-Galerkin operator.  All pointers are
// device memory owned by the op.  "ncp" is the cell count padded to a whole
// number of blocks; per-cell arrays are [field][ncp].
struct CGDev {
  int n_cell, ncp, n_dofs, n_free, n_blocks, n_shared;
  int nq;                 // quadrature points (<= 4 * MT of the kernel)
  int nbd_max;            // largest number of DoFs of one block
  int curved;             // geo holds one entry per rule point (see geo)
  int ncomp;              // components of the vector field (1: scalar), stored one after another
  int n_partials;         // partial sums per component
  double sigma;           // mass coefficient
  const void* geo;        // [7][ncp]: G00 G01 G02 G11 G12 G22 (= |detJ| J^-1 J^-T), |detJ|;
                          // curved: [ncp/16][7][nq][16] (16-cell tiles), the same per rule point
  const void* tab;        // basis table, layout chosen by the precision (see kernels.hip)
  const void* qw;         // [4*MT] quadrature weights, zero beyond nq
  const int* blk_priv_start;  // [n_blocks] first id of the block's private DoF range
  const int* blk_npriv;       // [n_blocks] private DoFs of the block
  const int* blk_nbd;         // [n_blocks] DoFs touched by the block
  const int* blk_other_off;   // [n_blocks] offset into other_gid / other_pslot
  const int* blk_ptr_off;     // [n_blocks] offset into slot_ptr
  const int* other_gid;       // global id of each non-private block DoF
  const int* other_pslot;     // partial-sum slot of each non-private block DoF (-1: constrained)
  const uint16_t* lidx;       // [ndof][ncp] block-local DoF index of (local node, cell)
  const uint16_t* pos;        // [ndof][ncp] LDS slot of (local node, cell), grouped by block DoF
  const uint16_t* slot_ptr;   // per block [nbd + 1] slot ranges of the block DoFs
  const int* sh_gid;          // [n_shared] global id of DoFs shared between blocks
  const int* sh_ptr;          // [n_shared + 1] their contiguous partial-sum ranges
  void* partials;             // [n_partials] scratch
};

// Device-side description of a discontinuous-Galerkin (SIPG) operator.
struct DGDev {
  int n_cell, ncp, n_face;
  int nq, nqf;
  int dirichlet;
  double sigma;
  const void* geo;        // [7][ncp]
  const void* tab;        // cell basis table
  const void* ftab;       // face basis table (reference face z = 0)
  const void* qw;         // [4*MT]
  const void* fw;         // [4*MTF] face weights
  const int* nb;          // [4][ncp] library id of the neighbour across local face f, -1 on the boundary
  const int* fid;         // [4][ncp] canonical face id
  const int* code;        // [4][ncp] own relabelling | neighbour relabelling << 8
  const void* fgeo;       // [8][4][ncp] b_own(3) b_nb(3) 2|F| tau
  const uint8_t* perm;    // [24][ndof] node permutation of each vertex relabelling
};

// Launchers (kernels.hip).  Return hipSuccess or the launch error.
// ev: NULL, or two events attached to the main kernel's dispatch
// (hipExtLaunchKernelGGL): its start and end timestamps.
hipError_t launch_cg(const CGDev& d, int prec, int ndof, int nq, int mode, const void* u, const void* g,
                     const void* kappa, void* out, void* dkappa, hipStream_t s, bool* supported,
                     hipEvent_t* ev);
hipError_t launch_dg(const DGDev& d, int prec, int ndof, int nq, int nqf, const void* u,
                     const void* kappa_cell, const void* kappa_face, void* v, hipStream_t s,
                     bool* supported, hipEvent_t* ev);
// SIPG coefficient gradients (dkappa_cell [nq][n_cell], dkappa_face
// [nqf][n_face], either may be NULL) of g^T A u; accumulate: add to them.
hipError_t launch_dg_grad(const DGDev& d, int prec, int ndof, int nq, int nqf, const void* u, const void* g,
                          void* dkc, void* dkf, bool accumulate, hipStream_t s, bool* supported);
// Device address of the fixed scratch array on the current device (resolved
// once per device, then cached); TETMF_NOALLOC_SCRATCH_BYTES long.
hipError_t noalloc_scratch(void** ptr);
hipError_t launch_layout(int prec, int to_user, const int* cell_perm, int n_cell, int nq,
                         const void* src, void* dst, hipStream_t s);

// Vector kernels used by the solver (kernels.hip).
hipError_t vec_fill(int prec, void* x, double value, int64_t n, hipStream_t s);
// Deterministic dot product: per-workgroup partial sums in FP64, reduced in
// fixed order by a single workgroup into *result (device FP64).
hipError_t vec_dot(int prec, const void* x, const void* y, int64_t n, double* partial, double* result,
                   hipStream_t s);
hipError_t vec_cast(int prec_src, const void* src, int prec_dst, void* dst, int64_t n, hipStream_t s);
// r = b - a (FP64)
hipError_t vec_sub(const double* b, const double* a, double* r, int64_t n, hipStream_t s);
// Fused Jacobi-PCG steps with device-resident FP64 scalars (kernels.hip).
// part: at least 3 * 512 doubles of partial sums.
// pcg_init: x = 0, r = rhs, z = dinv r, p = z (kept as it is when keep_p),
// *rz = r.z, *rr = r.r.
hipError_t pcg_init(int prec, const void* rhs, const void* dinv, void* x, void* r, void* z, void* p, double* part,
                    double* rz, double* rr, int64_t n, hipStream_t s, int keep_p = 0);
// One iteration after q = A p: alpha = rz_old / p.q, x += alpha p,
// r -= alpha q, z = dinv r, *rz_new = r.z, beta = rz_new / rz_old,
// p = z + beta p, *rr = r.r, and *pq_out = p.q when pq_out is not NULL.
// rz_old and rz_new must be distinct.
hipError_t pcg_iteration(int prec, void* x, void* r, void* z, void* p, const void* q, const void* dinv, double* part,
                         const double* rz_old, double* rz_new, double* rr, double* pq_out, int64_t n, hipStream_t s);
// One Chebyshev-Jacobi step (see tetmf_chebyshev): r = b - ax (ax NULL: r = b),
// d = cd d + cr dinv r (d not read unless d_read), x = (x_read ? x : 0) + d.
hipError_t cheb_step(int prec, const void* b, const void* ax, const void* dinv, void* d, void* x, double cd,
                     double cr, int d_read, int x_read, int64_t n, hipStream_t s);
// x_i in [-1, 1) from a fixed integer hash of i.
hipError_t vec_hash_fill(int prec, void* x, int64_t n, hipStream_t s);
hipError_t vec_recip(int prec, void* d, int64_t n, hipStream_t s);
hipError_t vec_axpy_f64(double* x, const void* d, int prec_d, int64_t n, hipStream_t s);

}  // namespace tetmf
