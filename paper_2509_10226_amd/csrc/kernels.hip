// HIP kernels for gfx950 (MI355X): matrix-free tetrahedral Galerkin operators.
//
// One operator application evaluates, for every cell e,
//     y += G_e^T E^T D_e E G_e u                              (eq. (5))
// and for SIPG additionally the face terms of eq. (7).  E (eq. (6)) is the
// table of reference gradients (and values) of the nodal basis at the
// quadrature points; it is identical for all cells, so 16 cells are batched
// into the N dimension of a matrix-core product, which is the GPU form of the
// paper's cells-batched matrix-matrix product (Sec. 2.4): the MFMA computes
//     T[(point, component), cell] = sum_j E[(point, component), j] U[j, cell]
// and, after the per-point operator D, integrates back with
//     V[j, cell] = sum_(point, component) E[(point, component), j] T[..., cell].
//
// Operand layout of the 16x16x4 matrix-core products (f64 and f32): lane l
// supplies A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16].  The
// accumulator element r of lane l holds output row  g + 4 r  (f64) or
// 4 g + r  (f32), g = l / 16, column l % 16 (measured on gfx950).  The rows
// of the interpolation tile are arranged so that lane group g, element r is
// component r of quadrature point 4 t + g: every lane then holds the three
// reference gradient components (and the value) of one point of one cell,
// the point operator D runs in registers, and the result is directly the B
// operand of the integration product (its K index is (point 4t+g, component r)).
//
// The E table lives in LDS ([point][component][NDOF+1], the odd stride keeps
// the 16 lanes that read one column on distinct banks).
#include "internal.h"

#include <algorithm>

namespace tetmf {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef d4 acc_t;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int g, int r) { return g + 4 * r; }
  __device__ static constexpr int row_g(int i) { return i & 3; }
  __device__ static constexpr int row_r(int i) { return i >> 2; }
};

template <>
struct Mfma<float> {
  typedef f4 acc_t;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int g, int r) { return 4 * g + r; }
  __device__ static constexpr int row_g(int i) { return i >> 2; }
  __device__ static constexpr int row_r(int i) { return i & 3; }
};

// T[(point 4t+g, comp r), cell] = sum_j tab[(point, comp), j] U[j, cell] for t < MT.
// U operand: lane supplies U[4s + g][cell c16] in ub[s].
template <typename T, int NDOF, int MT>
__device__ inline void interpolate(const T* __restrict__ s_tab, const T (&ub)[(NDOF + 3) / 4], int g, int c16,
                                   typename Mfma<T>::acc_t (&acc)[MT]) {
  using M = Mfma<T>;
  constexpr int NDP = NDOF + 1;
  constexpr int KS = (NDOF + 3) / 4;
  const int arow = 4 * M::row_g(c16) + M::row_r(c16);  // (point offset, component) of A row c16
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    acc[t] = typename M::acc_t{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int col = 4 * s + g;
      T a = (NDOF % 4 == 0 || col < NDOF) ? s_tab[(16 * t + arow) * NDP + col] : T(0);
      acc[t] = M::mma(a, ub[s], acc[t]);
    }
  }
}

// V[j, cell] = sum_(t, r) tab[(point 4t+g, comp r), j] T[t][r] for the dof tiles.
template <typename T, int NDOF, int MT>
__device__ inline void integrate(const T* __restrict__ s_tab, const typename Mfma<T>::acc_t (&tv)[MT], bool with_value,
                                 int g, int c16, typename Mfma<T>::acc_t (&v)[(NDOF + 15) / 16]) {
  using M = Mfma<T>;
  constexpr int NDP = NDOF + 1;
  constexpr int DT = (NDOF + 15) / 16;
#pragma unroll
  for (int m = 0; m < DT; ++m) {
    v[m] = typename M::acc_t{0, 0, 0, 0};
    const int col = 16 * m + c16;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (r == 3 && !with_value) continue;
        T a = (col < NDOF) ? s_tab[((4 * t + g) * 4 + r) * NDP + col] : T(0);
        v[m] = M::mma(a, tv[t][r], v[m]);
      }
    }
  }
}

// Block range of this workgroup: the blocks are split into 8 contiguous
// ranges, one per XCD (workgroups are dispatched round-robin over the XCDs),
// so that neighbouring blocks, which share DoFs, meet in the same L2.
__device__ inline void xcd_range(int n, int& first, int& last, int& stride) {
  const int nx = 8;
  const int x = blockIdx.x % nx;
  const int slot = blockIdx.x / nx;
  stride = gridDim.x / nx;
  const int lo = (int)((long long)n * x / nx);
  last = (int)((long long)n * (x + 1) / nx);
  first = lo + slot;
}

// ---------------------------------------------------------------------------
// continuous Galerkin: one workgroup pass per block of kBlockCells cells
//
// 1. stage the block's DoF values in LDS (private DoFs are a contiguous range
//    of the global vector; constrained DoFs read as zero: masked gather),
// 2. each wave gathers the B operands of its tiles from LDS,
// 3. interpolate, apply D, integrate (matrix cores), write the 16 x NDOF local
//    results to LDS slots grouped by block DoF,
// 4. sum every block DoF's slots in a fixed order; private DoFs are stored,
//    shared DoFs become partial sums that cg_combine adds in block order.
// Every sum has a fixed order, so the result is bitwise reproducible.

template <typename T, int NDOF, int MT, int MODE>
__global__ void __launch_bounds__(kThreads) cg_kernel(CGDev d, const T* __restrict__ u, const T* __restrict__ gin,
                                                      const T* __restrict__ kappa, T* __restrict__ out,
                                                      T* __restrict__ dk) {
  using M = Mfma<T>;
  typedef typename M::acc_t acc_t;
  constexpr int NDP = NDOF + 1;
  constexpr int NROW = MT * 16;
  constexpr int KS = (NDOF + 3) / 4;
  constexpr int DT = (NDOF + 15) / 16;
  constexpr bool BWD = MODE == MODE_BACKWARD;
  constexpr bool MF = MODE == MODE_APPLY || MODE == MODE_BACKWARD;
  extern __shared__ __align__(16) unsigned char smem[];
  T* s_tab = reinterpret_cast<T*>(smem);
  T* s_buf = s_tab + NROW * NDP;
  const T* tab = static_cast<const T*>(d.tab);
  for (int i = threadIdx.x; i < NROW * NDP; i += kThreads) s_tab[i] = tab[i];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int ncp = d.ncp, nc = d.n_cell;
  const T* geo = static_cast<const T*>(d.geo);
  const T* qw = static_cast<const T*>(d.qw);
  T* partials = static_cast<T*>(d.partials);
  const bool has_mass = d.sigma != 0.0;
  const T sigma = (T)d.sigma;
  const bool write_out = out != nullptr;
  T wq[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) wq[t] = qw[4 * t + g];
  int first, last, stride;
  xcd_range(d.n_blocks, first, last, stride);
  for (int b = first; b < last; b += stride) {
    __syncthreads();
    const int nbd = d.blk_nbd[b], npriv = d.blk_npriv[b], ps = d.blk_priv_start[b];
    const int oo = d.blk_other_off[b], po = d.blk_ptr_off[b];
    if (MF) {
      for (int k = threadIdx.x; k < nbd; k += kThreads) {
        int gi;
        bool ok = true;
        if (k < npriv) {
          gi = ps + k;
        } else {
          gi = d.other_gid[oo + k - npriv];
          ok = gi < d.n_free;
        }
        s_buf[k] = ok ? u[gi] : T(0);
        if (BWD) s_buf[nbd + k] = ok ? gin[gi] : T(0);
      }
    }
    __syncthreads();
    T ub[kTilesPerWave][KS];
    T gb[kTilesPerWave][BWD ? KS : 1];
    if (MF) {
#pragma unroll
      for (int tt = 0; tt < kTilesPerWave; ++tt) {
        const int cell = b * kBlockCells + (wave + tt * kWaves) * kTile + c16;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          const int j = 4 * s + g;
          const int l = (j < NDOF) ? d.lidx[j * ncp + cell] : 0;
          ub[tt][s] = (j < NDOF) ? s_buf[l] : T(0);
          if (BWD) gb[tt][s] = (j < NDOF) ? s_buf[nbd + l] : T(0);
        }
      }
    }
    __syncthreads();
    if (MF) {
#pragma unroll
      for (int tt = 0; tt < kTilesPerWave; ++tt) {
        const int cell = b * kBlockCells + (wave + tt * kWaves) * kTile + c16;
        const bool valid = cell < nc;
        const T G0 = geo[0 * ncp + cell], G1 = geo[1 * ncp + cell], G2 = geo[2 * ncp + cell];
        const T G3 = geo[3 * ncp + cell], G4 = geo[4 * ncp + cell], G5 = geo[5 * ncp + cell];
        const T adet = geo[6 * ncp + cell];
        acc_t acc[MT];
        interpolate<T, NDOF, MT>(s_tab, ub[tt], g, c16, acc);
        acc_t accg[BWD ? MT : 1];
        if (BWD) {
          T gtmp[KS];
#pragma unroll
          for (int s = 0; s < KS; ++s) gtmp[s] = gb[tt][BWD ? s : 0];
          acc_t tmp[MT];
          interpolate<T, NDOF, MT>(s_tab, gtmp, g, c16, tmp);
#pragma unroll
          for (int t = 0; t < MT; ++t) accg[BWD ? t : 0] = tmp[t];
        }
        acc_t tv[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          const int q = 4 * t + g;
          const bool qok = valid && q < d.nq;
          const T kap = qok ? (kappa ? kappa[(long)q * nc + cell] : T(1)) : T(0);
          const T s = kap * wq[t];
          if (BWD) {
            // dkappa = w_q grad_ref(u)^T G grad_ref(g)  (G already holds |det J|)
            const T ux = acc[t][0], uy = acc[t][1], uz = acc[t][2];
            const acc_t& gg = accg[BWD ? t : 0];
            const T gx = gg[0], gy = gg[1], gz = gg[2];
            const T dkv = wq[t] * (ux * (G0 * gx + G1 * gy + G2 * gz) + uy * (G1 * gx + G3 * gy + G4 * gz) +
                                   uz * (G2 * gx + G4 * gy + G5 * gz));
            if (dk && qok) dk[(long)q * nc + cell] = dkv;
          }
          const acc_t& src = BWD ? accg[BWD ? t : 0] : acc[t];
          const T x = src[0], y = src[1], z = src[2];
          tv[t][0] = s * (G0 * x + G1 * y + G2 * z);
          tv[t][1] = s * (G1 * x + G3 * y + G4 * z);
          tv[t][2] = s * (G2 * x + G4 * y + G5 * z);
          tv[t][3] = (has_mass && q < d.nq) ? sigma * wq[t] * adet * src[3] : T(0);
        }
        if (write_out) {
          acc_t v[DT];
          integrate<T, NDOF, MT>(s_tab, tv, has_mass, g, c16, v);
          if (valid) {
#pragma unroll
            for (int m = 0; m < DT; ++m)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int j = 16 * m + M::row(g, r);
                if (j < NDOF) s_buf[d.pos[j * ncp + cell]] = v[m][r];
              }
          }
        }
      }
    } else {
      // diagonal / load vector: one (cell, local node) pair per thread
      for (int idx = threadIdx.x; idx < kBlockCells * NDOF; idx += kThreads) {
        const int cl = idx % kBlockCells, j = idx / kBlockCells;
        const int cell = b * kBlockCells + cl;
        if (cell >= nc) continue;
        const T G0 = geo[0 * ncp + cell], G1 = geo[1 * ncp + cell], G2 = geo[2 * ncp + cell];
        const T G3 = geo[3 * ncp + cell], G4 = geo[4 * ncp + cell], G5 = geo[5 * ncp + cell];
        const T adet = geo[6 * ncp + cell];
        T acc = 0;
        for (int q = 0; q < d.nq; ++q) {
          const T w = qw[q];
          const T c = kappa ? kappa[(long)q * nc + cell] : T(1);
          const T x = s_tab[(q * 4 + 0) * NDP + j], y = s_tab[(q * 4 + 1) * NDP + j];
          const T z = s_tab[(q * 4 + 2) * NDP + j], val = s_tab[(q * 4 + 3) * NDP + j];
          if (MODE == MODE_DIAG) {
            acc += c * w *
                   (G0 * x * x + G3 * y * y + G5 * z * z + T(2) * (G1 * x * y + G2 * x * z + G4 * y * z));
            if (has_mass) acc += sigma * w * adet * val * val;
          } else {
            acc += w * adet * c * val;
          }
        }
        s_buf[d.pos[j * ncp + cell]] = acc;
      }
    }
    __syncthreads();
    if (write_out) {
      for (int k = threadIdx.x; k < nbd; k += kThreads) {
        const int p0 = d.slot_ptr[po + k], p1 = d.slot_ptr[po + k + 1];
        T s = 0;
        for (int p = p0; p < p1; ++p) s += s_buf[p];
        if (k < npriv) {
          out[ps + k] = s;
        } else {
          const int slot = d.other_pslot[oo + k - npriv];
          if (slot >= 0) partials[slot] = s;
        }
      }
    }
  }
}

// Shared DoFs: sum of the per-block partials in block order.  Constrained
// DoFs: identity rows (apply/backward), 1 (diagonal), 0 (load vector).
template <typename T, int MODE>
__global__ void __launch_bounds__(256) cg_combine(CGDev d, const T* __restrict__ u, T* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const T* part = static_cast<const T*>(d.partials);
  if (i < d.n_shared) {
    const int p0 = d.sh_ptr[i], p1 = d.sh_ptr[i + 1];
    T s = 0;
    for (int p = p0; p < p1; ++p) s += part[p];
    out[d.sh_gid[i]] = s;
  } else {
    const int c = i - d.n_shared;
    if (c < d.n_dofs - d.n_free) {
      const int gi = d.n_free + c;
      out[gi] = (MODE == MODE_APPLY || MODE == MODE_BACKWARD) ? u[gi] : (MODE == MODE_DIAG ? T(1) : T(0));
    }
  }
}

template <typename T, int NDOF, int MT, int MODE>
hipError_t launch_cg_t(const CGDev& d, const void* u, const void* g, const void* kappa, void* out, void* dk,
                       hipStream_t s, hipEvent_t* ev) {
  constexpr int NROW = MT * 16;
  constexpr int NDP = NDOF + 1;
  const int bufn = std::max(kBlockCells * NDOF, (MODE == MODE_BACKWARD ? 2 : 1) * d.nbd_max);
  const size_t lds = (size_t)(NROW * NDP + bufn) * sizeof(T);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  const int per_cu = lds <= 80 * 1024 ? 2 : 1;
  int grid = std::min(d.n_blocks, 256 * per_cu);
  grid = ((grid + 7) / 8) * 8;
  auto kern = cg_kernel<T, NDOF, MT, MODE>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (ev) (void)hipEventRecord(ev[0], s);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, d, (const T*)u, (const T*)g, (const T*)kappa, (T*)out,
                     (T*)dk);
  e = hipGetLastError();
  if (ev) (void)hipEventRecord(ev[1], s);
  if (e != hipSuccess || out == nullptr) return e;
  const int nfix = d.n_shared + (d.n_dofs - d.n_free);
  if (nfix > 0) {
    const T* src = (const T*)(MODE == MODE_BACKWARD ? g : u);
    hipLaunchKernelGGL((cg_combine<T, MODE>), dim3((nfix + 255) / 256), dim3(256), 0, s, d, src, (T*)out);
    e = hipGetLastError();
  }
  return e;
}

template <typename T, int NDOF, int MT>
hipError_t launch_cg_mode(const CGDev& d, int mode, const void* u, const void* g, const void* kappa, void* out,
                          void* dk, hipStream_t s, hipEvent_t* ev) {
  switch (mode) {
    case MODE_APPLY: return launch_cg_t<T, NDOF, MT, MODE_APPLY>(d, u, g, kappa, out, dk, s, ev);
    case MODE_BACKWARD: return launch_cg_t<T, NDOF, MT, MODE_BACKWARD>(d, u, g, kappa, out, dk, s, ev);
    case MODE_DIAG: return launch_cg_t<T, NDOF, MT, MODE_DIAG>(d, u, g, kappa, out, dk, s, ev);
    default: return launch_cg_t<T, NDOF, MT, MODE_LOAD>(d, u, g, kappa, out, dk, s, ev);
  }
}

template <typename T>
hipError_t launch_cg_shape(const CGDev& d, int ndof, int mt, int mode, const void* u, const void* g,
                           const void* kappa, void* out, void* dk, hipStream_t s, bool* supported, hipEvent_t* ev) {
  *supported = true;
  if (ndof == 4 && mt == 1) return launch_cg_mode<T, 4, 1>(d, mode, u, g, kappa, out, dk, s, ev);
  if (ndof == 10 && mt == 1) return launch_cg_mode<T, 10, 1>(d, mode, u, g, kappa, out, dk, s, ev);
  if (ndof == 10 && mt == 4) return launch_cg_mode<T, 10, 4>(d, mode, u, g, kappa, out, dk, s, ev);
  if (ndof == 20 && mt == 4) return launch_cg_mode<T, 20, 4>(d, mode, u, g, kappa, out, dk, s, ev);
  if (ndof == 20 && mt == 6) return launch_cg_mode<T, 20, 6>(d, mode, u, g, kappa, out, dk, s, ev);
  *supported = false;
  return hipSuccess;
}

hipError_t launch_cg(const CGDev& d, int prec, int ndof, int mt, int mode, const void* u, const void* g,
                     const void* kappa, void* out, void* dk, hipStream_t s, bool* supported, hipEvent_t* ev) {
  if (prec == PREC_F64) return launch_cg_shape<double>(d, ndof, mt, mode, u, g, kappa, out, dk, s, supported, ev);
  if (prec == PREC_F32) return launch_cg_shape<float>(d, ndof, mt, mode, u, g, kappa, out, dk, s, supported, ev);
  *supported = false;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// discontinuous Galerkin (SIPG), element-centric: each cell evaluates its
// cell term and, for each of its 4 faces, the face terms that test against
// its own basis functions (eq. (3) split by side).  Both traces are evaluated
// in a common frame: the face's vertices sorted by global id (a, b, c) are
// relabelled as reference vertices 0, 1, 2 and the opposite vertex as 3, for
// the own cell and for the neighbour.  Every face of every cell then uses the
// same face table (reference face z = 0) and the same point order; the
// relabelling is a permutation of the cell's nodes applied in the gather and
// in the accumulation.  Each cell writes only its own DoFs, so no
// synchronisation between cells is needed and the result is deterministic.
//
// Per face point (n = outward normal of the own cell, b = J_relabelled^-1 n so
// that d_n u = b . grad_ref u):
//   interior:  [[u]] = u- - u+,  {{d_n u}} = (d_n u- + d_n u+)/2
//   boundary (mirror u+ = -u-):  [[u]] = 2 u-, {{d_n u}} = d_n u-
//   value test:     omega kappa (tau [[u]] - {{d_n u}})
//   gradient test:  -omega kappa [[u]] / 2 * b_own

template <typename T, int NDOF, int MT, int MTF>
__global__ void __launch_bounds__(kThreads) dg_kernel(DGDev d, const T* __restrict__ u, const T* __restrict__ kc,
                                                      const T* __restrict__ kf, T* __restrict__ v) {
  using M = Mfma<T>;
  typedef typename M::acc_t acc_t;
  constexpr int NDP = NDOF + 1;
  constexpr int NROW = MT * 16;
  constexpr int NROWF = MTF * 16;
  constexpr int KS = (NDOF + 3) / 4;
  constexpr int DT = (NDOF + 15) / 16;
  extern __shared__ __align__(16) unsigned char smem[];
  T* s_tab = reinterpret_cast<T*>(smem);
  T* s_ftab = s_tab + NROW * NDP;
  T* s_out = s_ftab + NROWF * NDP;
  int* s_perm = reinterpret_cast<int*>(s_out + kWaves * kTile * NDOF);
  const T* tab = static_cast<const T*>(d.tab);
  const T* ftab = static_cast<const T*>(d.ftab);
  for (int i = threadIdx.x; i < NROW * NDP; i += kThreads) s_tab[i] = tab[i];
  for (int i = threadIdx.x; i < NROWF * NDP; i += kThreads) s_ftab[i] = ftab[i];
  for (int i = threadIdx.x; i < 24 * NDOF; i += kThreads) s_perm[i] = d.perm[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int ncp = d.ncp, nc = d.n_cell, nf = d.n_face;
  const T* geo = static_cast<const T*>(d.geo);
  const T* fgeo = static_cast<const T*>(d.fgeo);
  const T* qw = static_cast<const T*>(d.qw);
  const T* fw = static_cast<const T*>(d.fw);
  const bool has_mass = d.sigma != 0.0;
  const T sigma = (T)d.sigma;
  T wq[MT], fwq[MTF];
#pragma unroll
  for (int t = 0; t < MT; ++t) wq[t] = qw[4 * t + g];
#pragma unroll
  for (int t = 0; t < MTF; ++t) fwq[t] = fw[4 * t + g];
  T* so = s_out + wave * kTile * NDOF;
  // tiles of this wave: contiguous tile ranges per XCD
  const int ntiles = ncp / kTile;
  const int nx = 8, x = blockIdx.x % nx;
  const int per = (gridDim.x / nx) * kWaves;
  const int first = (int)((long long)ntiles * x / nx) + (blockIdx.x / nx) * kWaves + wave;
  const int last = (int)((long long)ntiles * (x + 1) / nx);
  for (int tile = first; tile < last; tile += per) {
    const int cell0 = tile * kTile;
    const int cell = cell0 + c16;
    const bool valid = cell < nc;
    // ---- cell term
    {
      T ub[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int j = 4 * s + g;
        ub[s] = (valid && j < NDOF) ? u[(long)cell * NDOF + j] : T(0);
      }
      const T G0 = geo[0 * ncp + cell], G1 = geo[1 * ncp + cell], G2 = geo[2 * ncp + cell];
      const T G3 = geo[3 * ncp + cell], G4 = geo[4 * ncp + cell], G5 = geo[5 * ncp + cell];
      const T adet = geo[6 * ncp + cell];
      acc_t acc[MT];
      interpolate<T, NDOF, MT>(s_tab, ub, g, c16, acc);
      acc_t tv[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const int q = 4 * t + g;
        const bool qok = valid && q < d.nq;
        const T s = (qok ? (kc ? kc[(long)q * nc + cell] : T(1)) : T(0)) * wq[t];
        const T xg = acc[t][0], yg = acc[t][1], zg = acc[t][2];
        tv[t][0] = s * (G0 * xg + G1 * yg + G2 * zg);
        tv[t][1] = s * (G1 * xg + G3 * yg + G4 * zg);
        tv[t][2] = s * (G2 * xg + G4 * yg + G5 * zg);
        tv[t][3] = (has_mass && qok) ? sigma * wq[t] * adet * acc[t][3] : T(0);
      }
      acc_t vv[DT];
      integrate<T, NDOF, MT>(s_tab, tv, has_mass, g, c16, vv);
#pragma unroll
      for (int m = 0; m < DT; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = 16 * m + M::row(g, r);
          if (j < NDOF) so[c16 * NDOF + j] = vv[m][r];
        }
    }
    // ---- face terms
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      const long fi = (long)f * ncp + cell;
      const int nbc = valid ? d.nb[fi] : -1;
      const int code = valid ? d.code[fi] : 0;
      const int fidv = valid ? d.fid[fi] : 0;
      const int ro = code & 255, rn = (code >> 8) & 255;
      const bool boundary = nbc < 0;
      const bool active = valid && (!boundary || d.dirichlet);
      T bo[3], bn[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        bo[k] = fgeo[((long)k * 4 + f) * ncp + cell];
        bn[k] = fgeo[((long)(3 + k) * 4 + f) * ncp + cell];
      }
      const T om = fgeo[((long)6 * 4 + f) * ncp + cell];
      const T tau = fgeo[((long)7 * 4 + f) * ncp + cell];
      T um[KS], up[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int j = 4 * s + g;
        um[s] = (valid && j < NDOF) ? u[(long)cell * NDOF + s_perm[ro * NDOF + j]] : T(0);
        up[s] = (!boundary && j < NDOF) ? u[(long)nbc * NDOF + s_perm[rn * NDOF + j]] : T(0);
      }
      acc_t am[MTF], ap[MTF];
      interpolate<T, NDOF, MTF>(s_ftab, um, g, c16, am);
      interpolate<T, NDOF, MTF>(s_ftab, up, g, c16, ap);
      acc_t tv[MTF];
#pragma unroll
      for (int t = 0; t < MTF; ++t) {
        const int q = 4 * t + g;
        const bool qok = active && q < d.nqf;
        const T s = (qok ? (kf ? kf[(long)q * nf + fidv] : T(1)) : T(0)) * fwq[t] * om;
        const T dnm = bo[0] * am[t][0] + bo[1] * am[t][1] + bo[2] * am[t][2];
        const T dnp = bn[0] * ap[t][0] + bn[1] * ap[t][1] + bn[2] * ap[t][2];
        const T jump = boundary ? T(2) * am[t][3] : am[t][3] - ap[t][3];
        const T avg = boundary ? dnm : T(0.5) * (dnm + dnp);
        const T cg = T(-0.5) * s * jump;
        tv[t][0] = cg * bo[0];
        tv[t][1] = cg * bo[1];
        tv[t][2] = cg * bo[2];
        tv[t][3] = s * (tau * jump - avg);
      }
      acc_t vf[DT];
      integrate<T, NDOF, MTF>(s_ftab, tv, true, g, c16, vf);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
      for (int m = 0; m < DT; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = 16 * m + M::row(g, r);
          if (j < NDOF) so[c16 * NDOF + s_perm[ro * NDOF + j]] += vf[m][r];
        }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    // ---- store the tile (contiguous 16 x NDOF block of the DG vector)
    for (int i = lane; i < kTile * NDOF; i += 64)
      if (cell0 + i / NDOF < nc) v[(long)cell0 * NDOF + i] = so[i];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

template <typename T, int NDOF, int MT, int MTF>
hipError_t launch_dg_t(const DGDev& d, const void* u, const void* kc, const void* kf, void* v, hipStream_t s,
                       hipEvent_t* ev) {
  constexpr int NDP = NDOF + 1;
  const size_t lds = (size_t)((MT + MTF) * 16 * NDP + kWaves * kTile * NDOF) * sizeof(T) + 24 * NDOF * sizeof(int);
  const int ntiles = d.ncp / kTile;
  int grid = std::min((ntiles + kWaves - 1) / kWaves, 256 * 2);
  grid = ((grid + 7) / 8) * 8;
  auto kern = dg_kernel<T, NDOF, MT, MTF>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (ev) (void)hipEventRecord(ev[0], s);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, d, (const T*)u, (const T*)kc, (const T*)kf, (T*)v);
  e = hipGetLastError();
  if (ev) (void)hipEventRecord(ev[1], s);
  return e;
}

template <typename T>
hipError_t launch_dg_shape(const DGDev& d, int ndof, int mt, int mtf, const void* u, const void* kc,
                           const void* kf, void* v, hipStream_t s, bool* supported, hipEvent_t* ev) {
  *supported = true;
  if (ndof == 4 && mt == 1 && mtf == 1) return launch_dg_t<T, 4, 1, 1>(d, u, kc, kf, v, s, ev);
  if (ndof == 10 && mt == 4 && mtf == 2) return launch_dg_t<T, 10, 4, 2>(d, u, kc, kf, v, s, ev);
  if (ndof == 20 && mt == 6 && mtf == 3) return launch_dg_t<T, 20, 6, 3>(d, u, kc, kf, v, s, ev);
  *supported = false;
  return hipSuccess;
}

hipError_t launch_dg(const DGDev& d, int prec, int ndof, int mt, int mtf, const void* u, const void* kc,
                     const void* kf, void* v, hipStream_t s, bool* supported, hipEvent_t* ev) {
  if (prec == PREC_F64) return launch_dg_shape<double>(d, ndof, mt, mtf, u, kc, kf, v, s, supported, ev);
  if (prec == PREC_F32) return launch_dg_shape<float>(d, ndof, mt, mtf, u, kc, kf, v, s, supported, ev);
  *supported = false;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// layout of per-point cell data: user [n_cell][nq] FP64 <-> library [nq][n_cell]

template <typename T>
__global__ void layout_kernel(int to_user, const int* __restrict__ perm, int nc, int nq, const void* src, void* dst) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= (long)nc * nq) return;
  const int q = (int)(i / nc), c = (int)(i % nc);
  const long user = (long)perm[c] * nq + q;
  if (!to_user)
    static_cast<T*>(dst)[i] = (T) static_cast<const double*>(src)[user];
  else
    static_cast<double*>(dst)[user] = (double)static_cast<const T*>(src)[i];
}

hipError_t launch_layout(int prec, int to_user, const int* cell_perm, int n_cell, int nq, const void* src, void* dst,
                         hipStream_t s) {
  const long n = (long)n_cell * nq;
  const int grid = (int)((n + 255) / 256);
  if (prec == PREC_F64)
    hipLaunchKernelGGL(layout_kernel<double>, dim3(grid), dim3(256), 0, s, to_user, cell_perm, n_cell, nq, src, dst);
  else
    hipLaunchKernelGGL(layout_kernel<float>, dim3(grid), dim3(256), 0, s, to_user, cell_perm, n_cell, nq, src, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// vector kernels for the conjugate-gradient solver

constexpr int kDotBlocks = 1024;

template <typename T>
__global__ void fill_kernel(T* x, double v, long n) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) x[i] = (T)v;
}

template <typename T>
__global__ void dot_partial(const T* __restrict__ x, const T* __restrict__ y, long n, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) s += (double)x[i] * (double)y[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void dot_final(const double* __restrict__ part, int np, double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

template <typename S, typename D>
__global__ void cast_kernel(const S* __restrict__ a, D* __restrict__ b, long n) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) b[i] = (D)a[i];
}

__global__ void sub_kernel(const double* __restrict__ b, const double* __restrict__ a, double* __restrict__ r, long n) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) r[i] = b[i] - a[i];
}

template <typename T>
__global__ void update_xr(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
                          const double* rz, const double* pq, long n) {
  const double alpha = *rz / *pq;
  const T a = (T)alpha;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    x[i] += a * p[i];
    r[i] -= a * q[i];
  }
}

template <typename T>
__global__ void precond_kernel(T* __restrict__ z, const T* __restrict__ r, const T* __restrict__ dinv, long n) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) z[i] = dinv[i] * r[i];
}

template <typename T>
__global__ void update_p(T* __restrict__ p, const T* __restrict__ z, const double* rz_new, const double* rz_old, long n) {
  const T beta = (T)(*rz_new / *rz_old);
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) p[i] = z[i] + beta * p[i];
}

template <typename T>
__global__ void recip_kernel(T* d, long n) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) d[i] = T(1) / d[i];
}

template <typename T>
__global__ void axpy64_kernel(double* __restrict__ x, const T* __restrict__ d, long n) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) x[i] += (double)d[i];
}

static int vgrid(long n) { return (int)std::min<long>((n + 255) / 256, 4096); }

#define TETMF_DISPATCH(prec, KERNEL, ...)                                                        \
  do {                                                                                           \
    if ((prec) == PREC_F64)                                                                      \
      hipLaunchKernelGGL(KERNEL<double>, dim3(vgrid(n)), dim3(256), 0, s, __VA_ARGS__);          \
    else                                                                                         \
      hipLaunchKernelGGL(KERNEL<float>, dim3(vgrid(n)), dim3(256), 0, s, __VA_ARGS__);           \
  } while (0)

hipError_t vec_fill(int prec, void* x, double value, int64_t n, hipStream_t s) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(fill_kernel<double>, dim3(vgrid(n)), dim3(256), 0, s, (double*)x, value, (long)n);
  else
    hipLaunchKernelGGL(fill_kernel<float>, dim3(vgrid(n)), dim3(256), 0, s, (float*)x, value, (long)n);
  return hipGetLastError();
}

hipError_t vec_dot(int prec, const void* x, const void* y, int64_t n, double* partial, double* result, hipStream_t s) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(dot_partial<double>, dim3(kDotBlocks), dim3(256), 0, s, (const double*)x, (const double*)y,
                       (long)n, partial);
  else
    hipLaunchKernelGGL(dot_partial<float>, dim3(kDotBlocks), dim3(256), 0, s, (const float*)x, (const float*)y,
                       (long)n, partial);
  hipLaunchKernelGGL(dot_final, dim3(1), dim3(256), 0, s, partial, kDotBlocks, result);
  return hipGetLastError();
}

hipError_t vec_cast(int ps, const void* src, int pd, void* dst, int64_t n, hipStream_t s) {
  if (ps == PREC_F64 && pd != PREC_F64)
    hipLaunchKernelGGL((cast_kernel<double, float>), dim3(vgrid(n)), dim3(256), 0, s, (const double*)src, (float*)dst,
                       (long)n);
  else if (ps != PREC_F64 && pd == PREC_F64)
    hipLaunchKernelGGL((cast_kernel<float, double>), dim3(vgrid(n)), dim3(256), 0, s, (const float*)src, (double*)dst,
                       (long)n);
  else if (ps == PREC_F64)
    hipLaunchKernelGGL((cast_kernel<double, double>), dim3(vgrid(n)), dim3(256), 0, s, (const double*)src,
                       (double*)dst, (long)n);
  else
    hipLaunchKernelGGL((cast_kernel<float, float>), dim3(vgrid(n)), dim3(256), 0, s, (const float*)src, (float*)dst,
                       (long)n);
  return hipGetLastError();
}

hipError_t vec_sub(const double* b, const double* a, double* r, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(sub_kernel, dim3(vgrid(n)), dim3(256), 0, s, b, a, r, (long)n);
  return hipGetLastError();
}

hipError_t pcg_update_xr(int prec, void* x, void* r, const void* p, const void* q, const double* rz, const double* pq,
                         int64_t n, hipStream_t s) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(update_xr<double>, dim3(vgrid(n)), dim3(256), 0, s, (double*)x, (double*)r, (const double*)p,
                       (const double*)q, rz, pq, (long)n);
  else
    hipLaunchKernelGGL(update_xr<float>, dim3(vgrid(n)), dim3(256), 0, s, (float*)x, (float*)r, (const float*)p,
                       (const float*)q, rz, pq, (long)n);
  return hipGetLastError();
}

hipError_t pcg_precond(int prec, void* z, const void* r, const void* dinv, int64_t n, hipStream_t s) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(precond_kernel<double>, dim3(vgrid(n)), dim3(256), 0, s, (double*)z, (const double*)r,
                       (const double*)dinv, (long)n);
  else
    hipLaunchKernelGGL(precond_kernel<float>, dim3(vgrid(n)), dim3(256), 0, s, (float*)z, (const float*)r,
                       (const float*)dinv, (long)n);
  return hipGetLastError();
}

hipError_t pcg_update_p(int prec, void* p, const void* z, const double* rz_new, const double* rz_old, int64_t n,
                        hipStream_t s) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(update_p<double>, dim3(vgrid(n)), dim3(256), 0, s, (double*)p, (const double*)z, rz_new, rz_old,
                       (long)n);
  else
    hipLaunchKernelGGL(update_p<float>, dim3(vgrid(n)), dim3(256), 0, s, (float*)p, (const float*)z, rz_new, rz_old,
                       (long)n);
  return hipGetLastError();
}

hipError_t vec_recip(int prec, void* d, int64_t n, hipStream_t s) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(recip_kernel<double>, dim3(vgrid(n)), dim3(256), 0, s, (double*)d, (long)n);
  else
    hipLaunchKernelGGL(recip_kernel<float>, dim3(vgrid(n)), dim3(256), 0, s, (float*)d, (long)n);
  return hipGetLastError();
}

hipError_t vec_axpy_f64(double* x, const void* d, int prec_d, int64_t n, hipStream_t s) {
  if (prec_d == PREC_F64)
    hipLaunchKernelGGL(axpy64_kernel<double>, dim3(vgrid(n)), dim3(256), 0, s, x, (const double*)d, (long)n);
  else
    hipLaunchKernelGGL(axpy64_kernel<float>, dim3(vgrid(n)), dim3(256), 0, s, x, (const float*)d, (long)n);
  return hipGetLastError();
}

}  // namespace tetmf
