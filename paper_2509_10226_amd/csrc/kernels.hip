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
// The E table lives in LDS ([point][component][NDP]: the DoF columns padded
// with zeros to 16, or to a multiple of 4, plus one; the odd stride keeps the
// 16 lanes that read one column on distinct banks).
#include "internal.h"
#include "lane_map.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>

#include "tetmf.h"

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
  __device__ static constexpr int row(int g, int r) { return lanes::acc_row(8, g, r); }
  __device__ static constexpr int row_g(int i) { return i & 3; }
  __device__ static constexpr int row_r(int i) { return i >> 2; }
};

template <>
struct Mfma<float> {
  typedef f4 acc_t;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int g, int r) { return lanes::acc_row(4, g, r); }
  __device__ static constexpr int row_g(int i) { return i >> 2; }
  __device__ static constexpr int row_r(int i) { return i & 3; }
};

// Sum of x over the four 16-lane rows of the wave, (r0 + r1) + (r2 + r3) in
// every lane, with the gfx950 lane-swap instructions (no LDS round trip).
// permlane16_swap(x, x) gives {x of rows 0,0,2,2; x of rows 1,1,3,3} and
// permlane32_swap(y, y) gives {y of the lower half twice; of the upper half}.
__device__ inline uint32_t row_swap16_lo(uint32_t x, uint32_t& hi) {
  const auto q = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  hi = q[1];
  return q[0];
}
__device__ inline uint32_t row_swap32_lo(uint32_t x, uint32_t& hi) {
  const auto q = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  hi = q[1];
  return q[0];
}
__device__ inline float sum_rows(float x) {
  uint32_t h16, h32;
  const float y = __uint_as_float(row_swap16_lo(__float_as_uint(x), h16)) + __uint_as_float(h16);
  return __uint_as_float(row_swap32_lo(__float_as_uint(y), h32)) + __uint_as_float(h32);
}
__device__ inline double sum_rows(double x) {
  const uint64_t b = __double_as_longlong(x);
  uint32_t h0, h1;
  const uint32_t l0 = row_swap16_lo((uint32_t)b, h0), l1 = row_swap16_lo((uint32_t)(b >> 32), h1);
  const double y = __longlong_as_double((long long)(((uint64_t)l1 << 32) | l0)) +
                   __longlong_as_double((long long)(((uint64_t)h1 << 32) | h0));
  const uint64_t c = __double_as_longlong(y);
  const uint32_t m0 = row_swap32_lo((uint32_t)c, h0), m1 = row_swap32_lo((uint32_t)(c >> 32), h1);
  return __longlong_as_double((long long)(((uint64_t)m1 << 32) | m0)) +
         __longlong_as_double((long long)(((uint64_t)h1 << 32) | h0));
}

// Layout of one 16-cell tile in the matrix-core registers.  Quadrature point
// p is handled by lane group p % 4 (as its k-th point, k = p / 4); item
// s = C k + c of a lane group is component c of its k-th point (components
// 0..2 are the reference gradient, component 3 the value when C = 4) and
// sits in accumulator element s % 4 of M-tile s / 4.  Every lane therefore
// owns whole points: the point operator runs in registers, and item s of all
// four lane groups together is exactly the B operand of K-step s of the
// integration product.  With C = 3 (no value needed) the 24-point rule fills
// 5 M-tiles instead of 6.
//
// The basis table in LDS is [NPTP points][C][NDP] (rows beyond the rule and
// columns beyond the DoFs are zero).  The integration runs the first 16 DoFs
// on the 16-row matrix-core product; the remaining NDOF - 16 DoFs (4 at
// p = 3), which would fill a second 16-row tile to a quarter, run in FP64 on
// the 4x4x4 four-block product, and in FP32 on the vector ALUs, summed over
// the four lane groups with cross-lane shuffles (the same fixed order in every
// lane, so the result is identical in all of them).
template <typename T, int NDOF, int NQ, int C>
struct Tile {
  using M = Mfma<T>;
  typedef typename M::acc_t acc_t;
  static constexpr int KP = (NQ + 3) / 4;
  static constexpr int NS = C * KP;
  static constexpr int MT = (NS + 3) / 4;
  static constexpr int KS = (NDOF + 3) / 4;
  // row length of the basis tables: NDOF + 1 in the global [point][4][row]
  // layout; in LDS the DoF columns are padded with zeros to 16 (at most 16
  // DoFs) or to a multiple of 4, plus one (an odd row stride), so that every
  // K step and every 16-row integration reads its missing columns as zeros
  // instead of under a per-lane predicate
  static constexpr int NDPG = NDOF + 1;
  static constexpr int NDP = (NDOF < 16 ? 16 : 4 * ((NDOF + 3) / 4)) + 1;
  static constexpr int NPT = 4 * KP;
  static constexpr int NMF = NDOF < 16 ? NDOF : 16;
  static constexpr int NVA = NDOF - NMF;
  // table rows reach the points of every item of the MT interpolation tiles
  // (items NS..4 MT - 1 of the last tile read zero rows, so no lane needs a
  // predicated load)
  static constexpr int NPTP = 4 * ((4 * MT - 1) / C + 1);
  static constexpr int TAB = NPTP * C * NDP;
  // B operand of the interpolation: lane group g supplies DoFs bdof(g, i), i < NB
  static constexpr int NB = KS;
  __device__ static constexpr int bdof(int g, int i) { return 4 * i + g; }
  // FP32 with four tail DoFs (P3): a second, 16-byte aligned copy of the tail
  // columns [row][4] after the table, so that each item's four values are one
  // 16-byte read at an immediate offset (the main table keeps its odd row
  // stride, which spreads its reads over the banks)
  static constexpr bool kTailTab = sizeof(T) == 4 && NVA == 4;
  static constexpr int TABA = (TAB + 3) / 4 * 4;
  static constexpr int TT = kTailTab ? NPTP * C * 4 : 0;
  // LDS bytes of the engine's tables (a multiple of 16)
  static constexpr int LDS_BYTES = ((TABA + TT) * (int)sizeof(T) + 15) / 16 * 16;

  // Tables from the global [NPT][4][NDOF + 1] layout into LDS (rows of
  // points NPT..NPTP - 1 zero).
  __device__ static inline void setup(unsigned char* lds, const T* __restrict__ gtab, int tid, int nt) {
    T* s_tab = reinterpret_cast<T*>(lds);
    for (int i = tid; i < TAB; i += nt) {
      const int col = i % NDP, c = (i / NDP) % C, p = i / (NDP * C);
      s_tab[i] = (p < NPT && col < NDOF) ? gtab[(p * 4 + c) * NDPG + col] : T(0);
    }
    if constexpr (kTailTab) {
      T* tt = s_tab + TABA;
      for (int i = tid; i < TT; i += nt) {
        const int r = i / 4, c = r % C, p = r / C;
        tt[i] = p < NPT ? gtab[(p * 4 + c) * NDPG + 16 + i % 4] : T(0);
      }
    }
  }

  __device__ static inline void interpolate(const unsigned char* lds, const T (&ub)[KS], int g, int c16,
                                            acc_t (&acc)[MT]) {
    interpolate(reinterpret_cast<const T*>(lds), ub, g, c16, acc);
  }
  __device__ static inline void integrate(const unsigned char* lds, const acc_t (&acc)[MT], int g, int c16, acc_t& v,
                                          T (&vv)[NDOF - (NDOF < 16 ? NDOF : 16) > 0 ? NDOF - (NDOF < 16 ? NDOF : 16) : 1]) {
    const T* s_tab = reinterpret_cast<const T*>(lds);
    integrate<kTailTab>(s_tab, acc, g, c16, v, vv, s_tab + TABA);
  }

  // acc[t] = rows (items) of M-tile t for the lane's cell column.
  __device__ static inline void interpolate(const T* __restrict__ s_tab, const T (&ub)[KS], int g, int c16,
                                            acc_t (&acc)[MT]) {
    const int gi = M::row_g(c16), ri = M::row_r(c16);
    // FP64 with a partly used last tile (NS % 4 items of 4, e.g. 2 at P3):
    // its items run on the 4x4x4 four-block product instead (see integrate
    // for the lane layout: with block b = cells 4b..4b+3, K = the four
    // DoFs of a step on the lane groups and rows = the lane groups, the B
    // operand is ub itself and lane group g receives the item of its own
    // points), at a quarter of the cost per item of the 16-row product.
    constexpr bool kSplitLast = sizeof(T) == 8 && NS % 4 != 0;
    constexpr int MTF = kSplitLast ? MT - 1 : MT;
#pragma unroll
    for (int t = 0; t < MTF; ++t) {
      const int s = 4 * t + ri;
      const int base = ((gi + 4 * (s / C)) * C + s % C) * NDP;
      acc[t] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const T a = s_tab[base + 4 * ks + g];  // zero columns beyond NDOF
        acc[t] = M::mma(a, ub[ks], acc[t]);
      }
    }
    if constexpr (kSplitLast) {
      const int gq = c16 & 3;  // row of A supplied by this lane: the item's lane group
      acc[MT - 1] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < NS % 4; ++r) {
        const int s = 4 * (MT - 1) + r;
        const int base = ((gq + 4 * (s / C)) * C + s % C) * NDP;
        T d = T(0);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const T a = s_tab[base + 4 * ks + g];
          d = __builtin_amdgcn_mfma_f64_4x4x4f64(a, ub[ks], d, 0, 0, 0);
        }
        acc[MT - 1][r] = d;
      }
    }
  }

  // v: DoFs 0..NMF-1 (element r of lane group g is DoF row(g, r));
  // vv[g] (lane groups g < NVA): DoF 16 + g of the lane's cell; the other
  // entries of vv are not meaningful.
  // TAILTAB: the FP32 tail reads its four values per item from tt (above)
  template <bool TAILTAB = false>
  __device__ static inline void integrate(const T* __restrict__ s_tab, const acc_t (&acc)[MT], int g, int c16,
                                          acc_t& v, T (&vv)[NVA > 0 ? NVA : 1], const T* __restrict__ tt = nullptr) {
    v = acc_t{0, 0, 0, 0};
    if constexpr (sizeof(T) == 8 && NDOF <= 12) {
      // FP64 with at most 12 DoFs (P1, P2): the 16-row product would be at
      // most three quarters full.  Instead, ceil(NDOF / 4) chains of the
      // 4x4x4 four-block product (lane layout as for the tail below): chain
      // r takes DoF 4r + (c16 & 3) as its A operand and delivers DoF 4r + g
      // to lane group g, which is exactly accumulator element r of the
      // 16-row layout (row g + 4r), at a quarter of its cost per chain.
#pragma unroll
      for (int r = 0; r < (NDOF + 3) / 4; ++r) {
        const int col = 4 * r + (c16 & 3);
        T t = T(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const T a = s_tab[((g + 4 * (s / C)) * C + s % C) * NDP + col];
          t = __builtin_amdgcn_mfma_f64_4x4x4f64(a, acc[s / 4][s % 4], t, 0, 0, 0);
        }
        v[r] = t;
      }
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const T a = s_tab[((g + 4 * (s / C)) * C + s % C) * NDP + c16];
        v = M::mma(a, acc[s / 4][s % 4], v);
      }
    }
    if constexpr (sizeof(T) == 8 && NVA == 4) {
      // DoFs 16..19 in FP64 on the 4x4x4 (four blocks) matrix-core product:
      // lane 16 k + 4 b + i supplies A[b][i][k] and B[b][k][i] and receives
      // D[b][k][i] (i, k < 4; measured on gfx950).  With block b = cells
      // 4b..4b+3, K = the four lane groups (the item's four points) and
      // rows = the four DoFs, the B operand is the item register itself and
      // lane group g receives DoF 16 + g of its cell: no cross-lane sums.
      T t = T(0);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const T a = s_tab[((g + 4 * (s / C)) * C + s % C) * NDP + 16 + (c16 & 3)];
        t = __builtin_amdgcn_mfma_f64_4x4x4f64(a, acc[s / 4][s % 4], t, 0, 0, 0);
      }
#pragma unroll
      for (int jj = 0; jj < NVA; ++jj) vv[jj] = t;
    } else if (NVA > 0) {
      T part[NVA > 0 ? NVA : 1];
#pragma unroll
      for (int jj = 0; jj < NVA; ++jj) part[jj] = T(0);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const T x = acc[s / 4][s % 4];
        const int row = (g + 4 * (s / C)) * C + s % C;
        if constexpr (TAILTAB) {
          static_assert(NVA == 4, "the aligned tail copy holds four columns");
          const float4 e = *reinterpret_cast<const float4*>(tt + 4 * row);
          part[0] += e.x * x;
          part[1] += e.y * x;
          part[2] += e.z * x;
          part[3] += e.w * x;
        } else {
          const T* e = s_tab + row * NDP + 16;
#pragma unroll
          for (int jj = 0; jj < NVA; ++jj) part[jj] += e[jj] * x;
        }
      }
#pragma unroll
      for (int jj = 0; jj < NVA; ++jj) vv[jj] = sum_rows(part[jj]);
    }
  }
};

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// BF16-operand engine: the same item layout as Tile<float> (the f32 16x16
// accumulator layout), but both products run as 16x16x32 BF16 matrix-core
// operations with FP32 accumulation.  Interpolation: one K-step covers all
// DoFs (lane group g supplies DoFs 8g..8g+7); integration: K-step ks takes
// items 8ks..8ks+7 of every lane group.  The operands are rounded to BF16
// (the table once at set-up, the DoF values and point values when they enter
// a product); the point operator and accumulation run in FP32.  DoFs 16..
// (4 at p = 3) are integrated by a second 16x16x32 chain on the same B
// operands whose A rows 4j hold DoF 16 + j (the other rows are zero), so
// that lane group j receives DoF 16 + j of its cell in accumulator element
// 0.  Tables in LDS: the interpolation A operands [MT][16][32], the
// integration A operands [KSI][16][32] and those of the tail DoFs, each lane
// reading 16 bytes.
template <int NDOF, int NQ, int C>
struct TileBF {
  using F = Tile<float, NDOF, NQ, C>;
  using M = Mfma<float>;
  typedef typename M::acc_t acc_t;
  static constexpr int KP = F::KP, NS = F::NS, MT = F::MT, NDP = F::NDPG, NPT = F::NPT;
  static constexpr int NMF = F::NMF, NVA = F::NVA;
  static constexpr int KSI = (NS + 7) / 8;
  static constexpr int NB = 8;
  __device__ static constexpr int bdof(int g, int i) { return 8 * g + i; }
  static constexpr int A_BYTES = MT * 16 * 32 * 2;
  static constexpr int B_BYTES = KSI * 16 * 32 * 2;
  static constexpr int LDS_BYTES = A_BYTES + (NVA > 0 ? 2 : 1) * B_BYTES;
  static_assert(NDOF <= 32, "one BF16 K-step covers at most 32 DoFs");
  static_assert(NVA <= 4, "the tail chain places at most 4 DoFs on rows 0, 4, 8, 12");

  __device__ static inline void setup(unsigned char* lds, const float* __restrict__ gtab, int tid, int nt) {
    __bf16* ta = reinterpret_cast<__bf16*>(lds);
    __bf16* tb = reinterpret_cast<__bf16*>(lds + A_BYTES);
    __bf16* tt = reinterpret_cast<__bf16*>(lds + A_BYTES + B_BYTES);
    for (int i = tid; i < MT * 16 * 32; i += nt) {
      const int kk = i % 32, row = (i / 32) % 16, t = i / 512;
      const int s = 4 * t + M::row_r(row), gi = M::row_g(row);
      const bool ok = s < NS && kk < NDOF;
      const float e = ok ? gtab[((gi + 4 * (s / C)) * 4 + s % C) * NDP + kk] : 0.0f;
      ta[i] = (__bf16)e;
    }
    for (int i = tid; i < KSI * 16 * 32; i += nt) {
      const int kk = i % 32, row = (i / 32) % 16, ks = i / 512;
      const int gk = kk / 8, s = 8 * ks + kk % 8;
      const bool ok = s < NS && row < NMF;
      const float e = ok ? gtab[((gk + 4 * (s / C)) * 4 + s % C) * NDP + row] : 0.0f;
      tb[i] = (__bf16)e;
      if (NVA > 0) {
        // tail DoF 16 + row / 4 on rows 0, 4, 8, 12
        const bool okt = s < NS && row % 4 == 0 && row / 4 < NVA;
        const float et = okt ? gtab[((gk + 4 * (s / C)) * 4 + s % C) * NDP + 16 + row / 4] : 0.0f;
        tt[i] = (__bf16)et;
      }
    }
  }

  __device__ static inline void interpolate(const unsigned char* lds, const float (&ub)[NB], int g, int c16,
                                            acc_t (&acc)[MT]) {
    const bf8* ta = reinterpret_cast<const bf8*>(lds);
    bf8 b;
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = (__bf16)ub[i];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const bf8 a = ta[(t * 16 + c16) * 4 + g];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc_t{0, 0, 0, 0}, 0, 0, 0);
    }
  }

  __device__ static inline void integrate(const unsigned char* lds, const acc_t (&acc)[MT], int g, int c16, acc_t& v,
                                          float (&vv)[NVA > 0 ? NVA : 1]) {
    const bf8* tb = reinterpret_cast<const bf8*>(lds + A_BYTES);
    const bf8* tt = reinterpret_cast<const bf8*>(lds + A_BYTES + B_BYTES);
    v = acc_t{0, 0, 0, 0};
    acc_t vt = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KSI; ++ks) {
      bf8 b;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int s = 8 * ks + e;
        b[e] = (__bf16)(s < NS ? acc[s < NS ? s / 4 : 0][s % 4] : 0.0f);
      }
      const bf8 a = tb[(ks * 16 + c16) * 4 + g];
      v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, v, 0, 0, 0);
      if (NVA > 0) {
        const bf8 at = tt[(ks * 16 + c16) * 4 + g];
        vt = __builtin_amdgcn_mfma_f32_16x16x32_bf16(at, b, vt, 0, 0, 0);
      }
    }
#pragma unroll
    for (int jj = 0; jj < (NVA > 0 ? NVA : 1); ++jj) vv[jj] = vt[0];
  }
};

template <typename T, int NDOF, int NQ, int C, bool BF>
struct EngineSel {
  typedef Tile<T, NDOF, NQ, C> type;
};
template <int NDOF, int NQ, int C>
struct EngineSel<float, NDOF, NQ, C, true> {
  typedef TileBF<NDOF, NQ, C> type;
};

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

// Entries staged (or reduced) per thread between two waits for memory.
constexpr int kStageUnroll = 4;

// Workgroups of a persistent launch: as many as are resident at once on the
// device (occupancy from the kernel's registers and LDS), a multiple of the 8
// XCDs, and no more than there is work.
static int persistent_grid(const void* kern, size_t lds, int work) {
  int dev = 0, cus = 256, per_cu = 1;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int grid = std::min(work, cus * per_cu);
  return std::max(8, ((grid + 7) / 8) * 8);
}

// ---------------------------------------------------------------------------
// continuous Galerkin: one workgroup pass per block of kBlockCells cells
//
// 1. stage the block's DoF values in LDS (private DoFs are a contiguous range
//    of the global vector; constrained DoFs read as zero: masked gather) and
//    the block's local DoF indices of every (cell, node),
// 2. each wave gathers the B operands of its tiles from LDS,
// 3. interpolate, apply D, integrate, write the 16 x NDOF local results to
//    LDS slots grouped by block DoF,
// 4. sum every block DoF's slots in a fixed order; private DoFs are stored,
//    shared DoFs become partial sums that cg_combine adds in block order.
// Every sum has a fixed order, so the result is bitwise reproducible.

// Load base[off / sizeof(X)] with a wave-uniform 64-bit base and a per-lane
// 32-bit byte offset, the form the global loads with a scalar base address
// take (no 64-bit address arithmetic per lane).
template <typename X>
__device__ inline X load_at(const X* __restrict__ base, uint32_t byte_off) {
  return *reinterpret_cast<const X*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Thread index hidden from loop-invariant code motion: values derived from it
// inside a phase are not kept live across the other phases of the block loop
// (the compute phase needs every register for the matrix-core tiles).
__device__ inline int phase_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Sum the slots of every block DoF (fixed order) and store them.
template <typename T>
__device__ inline void cg_reduce(const CGDev& d, const T* __restrict__ s_slot, int nbd, int npriv, int ps, int oo,
                                 int po, T* __restrict__ out, T* __restrict__ partials) {
  const int nother = nbd - npriv;
  for (int k0 = 0; k0 < nbd; k0 += kStageUnroll * kThreads) {
    int p0[kStageUnroll], p1[kStageUnroll], dst[kStageUnroll];
#pragma unroll
    for (int i = 0; i < kStageUnroll; ++i) {
      const int k = k0 + i * kThreads + threadIdx.x;
      const bool in = k < nbd;
      const int kc = min(k, nbd);
      const int a = d.slot_ptr[po + kc], bnd = d.slot_ptr[po + min(kc + 1, nbd)];
      const int ps_ = d.other_pslot[oo + min(max(k - npriv, 0), max(nother - 1, 0))];
      p0[i] = in ? a : 0;
      p1[i] = in ? bnd : 0;
      dst[i] = !in ? -1 : (k < npriv ? -2 : ps_);
    }
#pragma unroll
    for (int i = 0; i < kStageUnroll; ++i) {
      const int k = k0 + i * kThreads + threadIdx.x;
      // two slots per step (same left-to-right order of the sum)
      T s = 0;
      int p = p0[i];
      for (; p + 1 < p1[i]; p += 2) {
        s += s_slot[p];
        s += s_slot[p + 1];
      }
      if (p < p1[i]) s += s_slot[p];
      if (dst[i] == -2)
        out[ps + k] = s;
      else if (dst[i] >= 0)
        partials[dst[i]] = s;
    }
  }
}

// Geometry of one rule point of the lane's cell for curved cells: value
// (c, q) of the cell's 16-cell tile of the geometry ([ncp / 16][7][NQ][16]),
// q = g + 4k clamped to the rule, read with the tile as the base and a
// 32-bit offset inside it.
// dep: a value computed just before; the offset passes through an empty asm
// that depends on it, so the loads are issued there and not hoisted (the
// matrix-core tiles need the registers).
// G[7] receives the coefficient at the point (1 without one; cc: the cell
// clamped to the mesh).
template <typename T, int NQ, int C>
__device__ inline void point_geo(const T* __restrict__ geo, int ncp, const T* __restrict__ kappa, int nc, int k,
                                 int g, int cell, int cc, T dep, T (&G)[8]) {
  const int q = min(g + 4 * k, NQ - 1);
  // geometry: the cell's 16-cell tile (the geometry is padded to whole
  // blocks) as the base and the point and cell inside it as the offset
  uint32_t off = (uint32_t)lanes::curved_geo_index(NQ, 0, q, cell & 15) * (uint32_t)sizeof(T);
  // coefficient: tile base of the clamped cell and an offset inside its tile
  uint32_t kof = (uint32_t)lanes::cell_data_index(NQ, q, cc & 15) * (uint32_t)sizeof(T);
  asm volatile("" : "+v"(off), "+v"(kof) : "v"(dep));
  const T* gt = geo + lanes::curved_geo_index(NQ, 0, 0, cell & ~15);
  (void)ncp;
#pragma unroll
  for (int c = 0; c < (C == 4 ? 7 : 6); ++c) G[c] = load_at(gt + c * NQ * 16, off);
  if (C != 4) G[6] = T(0);
  G[7] = kappa ? load_at(kappa + lanes::cell_data_index(NQ, 0, cc & ~15), kof) : T(1);
  (void)nc;
}

// NCOMP > 1: a vector field of NCOMP components without coupling (Sec. 3.2),
// stored component by component; each block stages its local indices once
// and runs stage / tiles / reduce per component (the LDS holds one
// component at a time), re-reading the cell data from cache.
// Register budget: four waves per SIMD (two workgroups per CU, the LDS
// limit of the forward kernels).  The FP64 backward at P3 stages u and g
// (about 90 KB of LDS per workgroup at the 64^3 x 6 mesh), so one workgroup
// fits per CU and two waves per SIMD lose nothing; the budget then allows 256
// registers instead of spilling at 128.  Curved FP64 cells take two waves
// too: they request every point's geometry of a tile at once (see
// CurvAhead), and the bytes in flight per SIMD outweigh the halved occupancy.
template <typename T, int NDOF, int MODE, bool CURV>
struct MinWaves {
  static constexpr int value =
      ((sizeof(T) == 8 && NDOF == 20 && MODE == MODE_BACKWARD) || (CURV && sizeof(T) == 8)) ? 2 : 4;
};

// Curved cells read a geometry and a coefficient per point.  FP64: all of a
// tile's points are requested before its interpolation (588 -> 582 us at
// 64^3 x 6), except in the Helmholtz backward, which would spill with them.  FP32: one point at a
// time, each request tied to the previous point's result (all at once:
// 330 -> 363 us).
template <typename T, bool CURV>
struct CurvAhead {
  static constexpr bool value = CURV && sizeof(T) == 8;
};

template <typename T, int NDOF, int NQ, int C, int MODE, bool BF, bool CURV, int NCOMP>
__global__ void __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(MinWaves<T, NDOF, MODE, CURV>::value, 8))) cg_kernel(CGDev d, const T* __restrict__ u, const T* __restrict__ gin, const T* __restrict__ kappa,
          T* __restrict__ out, T* __restrict__ dk) {
  using TL = typename EngineSel<T, NDOF, NQ, C, BF>::type;
  using M = Mfma<T>;
  typedef typename M::acc_t acc_t;
  constexpr int NB = TL::NB, KP = TL::KP, MT = TL::MT;
  constexpr bool BWD = MODE == MODE_BACKWARD;
  extern __shared__ __align__(16) unsigned char smem[];
  // LDS: engine tables | weights | block slots | staged DoF values | local indices
  unsigned char* s_eng = smem;
  T* s_qw = reinterpret_cast<T*>(smem + TL::LDS_BYTES);
  T* s_slot = s_qw + TL::NPT;
  T* s_u = s_slot + kBlockCells * NDOF;
  uint16_t* s_lidx = reinterpret_cast<uint16_t*>(s_u + (BWD ? 2 : 1) * d.nbd_max);
  TL::setup(s_eng, static_cast<const T*>(d.tab), threadIdx.x, kThreads);
  for (int i = threadIdx.x; i < TL::NPT; i += kThreads) s_qw[i] = static_cast<const T*>(d.qw)[i];
  const int ncp = d.ncp, nc = d.n_cell;
  const T* geo = static_cast<const T*>(d.geo);
  const T sigma = (T)d.sigma;
  const bool write_out = out != nullptr;
  int first, last, stride;
  xcd_range(d.n_blocks, first, last, stride);
  for (int b = first; b < last; b += stride) {
    const int nbd = d.blk_nbd[b], npriv = d.blk_npriv[b], ps = d.blk_priv_start[b];
    const int oo = d.blk_other_off[b], po = d.blk_ptr_off[b];
    // one pass per component (a scalar field: one pass with comp = 0)
    auto comp_pass = [&](const int comp) {
      const T* uc = u + (long)comp * d.n_dofs;
      const T* gc = BWD ? gin + (long)comp * d.n_dofs : gin;
      T* oc = write_out ? out + (long)comp * d.n_dofs : out;
      __syncthreads();  // previous block's (component's) slots, staged values and indices are consumed
      {
        // curved cells: thread index re-derived per block, so that the staging
        // addresses are not kept live across the compute phase (which needs
        // the registers for the per-point geometry; the straight kernels are
        // faster with them kept)
        const unsigned st = CURV ? (unsigned)phase_tid() : threadIdx.x;
        // block-local indices: [NDOF][kBlockCells] uint16, copied as 32-bit words
        const uint32_t* src = reinterpret_cast<const uint32_t*>(d.lidx);
        uint32_t* dstw = reinterpret_cast<uint32_t*>(s_lidx);
        constexpr int W = NDOF * kBlockCells / 2;
        uint32_t wv[(W + kThreads - 1) / kThreads];
        if (comp == 0) {
#pragma unroll
          for (int i = 0; i < (W + kThreads - 1) / kThreads; ++i) {
            const int w = i * kThreads + st;
            const int j = (2 * w) / kBlockCells, cl = (2 * w) % kBlockCells;
            // word (j ncp + b kBlockCells + cl) / 2: block base + 32-bit byte offset
            wv[i] = w < W ? load_at(src + (long)b * (kBlockCells / 2),
                                    2u * ((uint32_t)j * (uint32_t)ncp + (uint32_t)cl))
                          : 0u;
          }
        }
        // DoF values: all index loads first, then all value loads (clamped
        // indices keep every load in bounds, so no load needs a branch; the
        // other-DoF lists carry one padding entry for blocks without any)
        const int nother = nbd - npriv;
        for (int k0 = 0; k0 < nbd; k0 += kStageUnroll * kThreads) {
          int gi[kStageUnroll];
          bool ok[kStageUnroll];
#pragma unroll
          for (int i = 0; i < kStageUnroll; ++i) {
            const int k = k0 + i * kThreads + st;
            const int oi = min(max(k - npriv, 0), max(nother - 1, 0));
            const int og = load_at(d.other_gid + oo, (uint32_t)oi * 4u);
            gi[i] = (k < npriv) ? ps + k : og;
            ok[i] = k < nbd && (k < npriv || og < d.n_free);
          }
          T uv[kStageUnroll], gv[kStageUnroll];
#pragma unroll
          for (int i = 0; i < kStageUnroll; ++i) {
            const uint32_t src_o = (uint32_t)(ok[i] ? gi[i] : 0) * (uint32_t)sizeof(T);
            uv[i] = load_at(uc, src_o);
            if (BWD) gv[i] = load_at(gc, src_o);
            uv[i] = ok[i] ? uv[i] : T(0);
            if (BWD) gv[i] = ok[i] ? gv[i] : T(0);
          }
#pragma unroll
          for (int i = 0; i < kStageUnroll; ++i) {
            const int k = k0 + i * kThreads + st;
            if (k < nbd) {
              s_u[k] = uv[i];
              if (BWD) s_u[d.nbd_max + k] = gv[i];
            }
          }
        }
        if (comp == 0) {
#pragma unroll
          for (int i = 0; i < (W + kThreads - 1) / kThreads; ++i) {
            const int w = i * kThreads + st;
            if (w < W) dstw[w] = wv[i];
          }
        }
      }
      __syncthreads();
#pragma unroll 1
      for (int tt = 0; tt < kTilesPerWave; ++tt) {
        // lane coordinates re-derived per tile (not held across the block loop)
        const int tid = phase_tid();
        const int lane = tid & 63, wave = tid >> 6;
        const int g = lane >> 4, c16 = lane & 15;
        const int cl = (wave + tt * kWaves) * kTile + c16;
        const int cell = b * kBlockCells + cl;
        const bool valid = cell < nc;
        // per-cell arrays: row base (uniform) + 32-bit lane offset
        // straight cells: G and |det J| of the cell (curved: per point below)
        T Gc[7];
        if constexpr (!CURV) {
          const uint32_t coff = (uint32_t)cell * (uint32_t)sizeof(T);
#pragma unroll
          for (int c = 0; c < 6; ++c) Gc[c] = load_at(geo + c * (long)ncp, coff);
          Gc[6] = (C == 4) ? load_at(geo + 6 * (long)ncp, coff) : T(0);
        }
        // coefficient at this lane's points q = g + 4k (point q of the cell's
        // 16-cell tile of the per-point data),
        // from a clamped (always valid) address and masked afterwards
        T kq[KP];
        if (CURV) {
          // loaded with the per-point geometry
        } else if (kappa) {
          const int cc = valid ? cell : nc - 1;
          // the tile's contiguous run (base) and the lane's point and cell
          // inside it (a 32-bit offset below 16 NQ sizeof(T))
          const T* kt = kappa + lanes::cell_data_index(NQ, 0, cc & ~15);
#pragma unroll
          for (int k = 0; k < KP; ++k)
            kq[k] = load_at(kt, (uint32_t)lanes::cell_data_index(NQ, 4 * k + lanes::kappa_lane_row(NQ, g, k), cc & 15) *
                                    (uint32_t)sizeof(T));
        } else {
#pragma unroll
          for (int k = 0; k < KP; ++k) kq[k] = T(1);
        }
        // LDS slots of the lane's result rows; straight cells request them
        // with the cell data, curved FP64 cells after the point loop (they are
        // needed only for the slot writes, and the per-point geometry needs
        // the registers before that: 622 -> 590 us at 64^3 x 6; FP32 has the
        // registers and keeps the early request)
        constexpr bool kLateSlots = CURV && sizeof(T) == 8;
        uint16_t pv[4 + TL::NVA];
        auto load_slots = [&]() {
          // row(g, r) = row(g, 0) + row(0, r): lane part and uniform part
          const uint32_t pof = ((uint32_t)M::row(g, 0) * (uint32_t)ncp + (uint32_t)cell) * 2u;
          // rows beyond the cell's DoFs (fewer than 16 at p <= 2) have no slot
#pragma unroll
          for (int r = 0; r < 4; ++r)
            pv[r] = lanes::pos_row(sizeof(T), NDOF, g, r) >= 0 ? load_at(d.pos + (long)M::row(0, r) * ncp, pof)
                                                               : uint16_t(0);
          if constexpr (TL::NVA > 0)
            pv[4] = load_at(d.pos + 16 * (long)ncp,
                            ((uint32_t)(lanes::pos_tail_row(NDOF, g) - 16) * (uint32_t)ncp + (uint32_t)cell) * 2u);
        };
        if (!kLateSlots && write_out) load_slots();
        T ub[NB];
        T gb[BWD ? NB : 1];
#pragma unroll
        for (int ks = 0; ks < NB; ++ks) {
          // operand rows beyond the cell's DoFs read a valid row and are
          // zeroed afterwards (no branch around the loads)
          const int j = TL::bdof(g, ks);
          const int l = s_lidx[lanes::operand_row(NDOF, j) * kBlockCells + cl];
          const T x = s_u[l];
          ub[ks] = j < NDOF ? x : T(0);
          if (BWD) {
            const T y = s_u[d.nbd_max + l];
            gb[BWD ? ks : 0] = j < NDOF ? y : T(0);
          }
        }
        // (not for the curved Helmholtz backward, which holds the second
        // interpolation's four values per item as well: all points' geometry
        // at once would spill there)
        constexpr bool kAhead = CurvAhead<T, CURV>::value && !(BWD && C == 4);
        T Gpre[kAhead ? KP : 1][8];
        if constexpr (kAhead) {
          const int cc = valid ? cell : nc - 1;
#pragma unroll
          for (int k = 0; k < KP; ++k) point_geo<T, NQ, C>(geo, ncp, kappa, nc, k, g, cell, cc, T(0), Gpre[k]);
        }
        acc_t acc[MT];
        // matrix-core section of the tile at raised wave priority: the
        // arbiter then prefers the waves issuing products over those in
        // their staging, gather or reduction code
        __builtin_amdgcn_s_setprio(1);
        TL::interpolate(s_eng, ub, g, c16, acc);
        acc_t accg[BWD ? MT : 1];
        if (BWD) {
          T gtmp[NB];
#pragma unroll
          for (int ks = 0; ks < NB; ++ks) gtmp[ks] = gb[BWD ? ks : 0];
          acc_t tmp[MT];
          TL::interpolate(s_eng, gtmp, g, c16, tmp);
#pragma unroll
          for (int t = 0; t < MT; ++t) accg[BWD ? t : 0] = tmp[t];
        }
        // point operator D in registers: item s = C k + c at acc[s / 4][s % 4].
        // Curved FP32 cells: the geometry of point k is requested once point
        // k - 1 is done (FP64: all points requested above).
        const int ccell = valid ? cell : nc - 1;
        // per-tile copies of the bases, so that the row addresses derived from
        // them are not hoisted out of the block loop (36 of them at P3)
        const T* geot = geo;
        const T* kapt = kappa;
        if constexpr (CURV) asm volatile("" : "+s"(geot), "+s"(kapt));
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          T Gk[8];
          if constexpr (kAhead) {
#pragma unroll
            for (int c = 0; c < 8; ++c) Gk[c] = Gpre[kAhead ? k : 0][c];
          } else if constexpr (CURV) {
            const int ip = C * (k > 0 ? k - 1 : 0);
            point_geo<T, NQ, C>(geot, ncp, kapt, nc, k, g, cell, ccell, acc[ip / 4][ip % 4], Gk);
          } else {
#pragma unroll
            for (int c = 0; c < 7; ++c) Gk[c] = Gc[c];
            Gk[7] = kq[k];
          }
          const T G0 = Gk[0], G1 = Gk[1], G2 = Gk[2], G3 = Gk[3], G4 = Gk[4], G5 = Gk[5], adet = Gk[6];
          const int q = g + 4 * k;
          const T w = s_qw[q];
          const bool qok = valid && q < NQ;
          // straight cells leave the products unmasked (padded points have
          // zero weight and zero table rows, padded cells' results are never
          // stored): 70.2 -> 68.8 us for P2 Helmholtz at 48^3 x 6; curved
          // cells keep the mask (it holds their register budget)
          const T s = CURV ? (qok ? Gk[7] * w : T(0)) : Gk[7] * w;
          const int i0 = C * k;
          T x, y, z, val = T(0);
          if (BWD) {
            const T ux = acc[(i0) / 4][(i0) % 4], uy = acc[(i0 + 1) / 4][(i0 + 1) % 4];
            const T uz = acc[(i0 + 2) / 4][(i0 + 2) % 4];
            x = accg[BWD ? (i0) / 4 : 0][(i0) % 4];
            y = accg[BWD ? (i0 + 1) / 4 : 0][(i0 + 1) % 4];
            z = accg[BWD ? (i0 + 2) / 4 : 0][(i0 + 2) % 4];
            if constexpr (C == 4) val = accg[BWD ? (i0 + 3) / 4 : 0][(i0 + 3) % 4];
            // dkappa = w_q grad_ref(u)^T G grad_ref(g)  (G already holds |det J|)
            const T dkv = w * (ux * (G0 * x + G1 * y + G2 * z) + uy * (G1 * x + G3 * y + G4 * z) +
                               uz * (G2 * x + G4 * y + G5 * z));
            // vector fields: the sum over the components, in component order
            if (dk && qok) {
              const long di = lanes::cell_data_index(NQ, q, cell);
              if (comp == 0)
                dk[di] = dkv;
              else
                dk[di] += dkv;
            }
          } else {
            x = acc[(i0) / 4][(i0) % 4];
            y = acc[(i0 + 1) / 4][(i0 + 1) % 4];
            z = acc[(i0 + 2) / 4][(i0 + 2) % 4];
            if constexpr (C == 4) val = acc[(i0 + 3) / 4][(i0 + 3) % 4];
          }
          acc[(i0) / 4][(i0) % 4] = s * (G0 * x + G1 * y + G2 * z);
          acc[(i0 + 1) / 4][(i0 + 1) % 4] = s * (G1 * x + G3 * y + G4 * z);
          acc[(i0 + 2) / 4][(i0 + 2) % 4] = s * (G2 * x + G4 * y + G5 * z);
          if constexpr (C == 4)
            acc[(i0 + 3) / 4][(i0 + 3) % 4] = CURV ? (qok ? sigma * w * adet * val : T(0)) : sigma * w * adet * val;
        }
        if (write_out) {
          if (kLateSlots) load_slots();
          acc_t v;
          T vv[TL::NVA > 0 ? TL::NVA : 1];
          TL::integrate(s_eng, acc, g, c16, v, vv);
          if (valid) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (lanes::pos_row(sizeof(T), NDOF, g, r) >= 0) s_slot[pv[r]] = v[r];
            if constexpr (TL::NVA > 0) {
              T mine = vv[0];
#pragma unroll
              for (int jj = 1; jj < (TL::NVA > 0 ? TL::NVA : 1); ++jj) mine = (g == jj) ? vv[jj] : mine;
              if (g < TL::NVA) s_slot[pv[4]] = mine;
            }
          }
        }
        __builtin_amdgcn_s_setprio(0);
      }
      __syncthreads();
      if (write_out)
        cg_reduce<T>(d, s_slot, nbd, npriv, ps, oo, po, oc, static_cast<T*>(d.partials) + (long)comp * d.n_partials);
    };
    if constexpr (NCOMP == 1) {
      comp_pass(0);
    } else {
#pragma unroll 1
      for (int comp = 0; comp < NCOMP; ++comp) comp_pass(comp);
    }
  }
}

// Diagonal and load vector (setup-time work, vector ALUs): one (cell, local
// node) pair per thread, same slots and fixed-order block reduction.
template <typename T, int NDOF, int NQ, int MODE, bool CURV>
__global__ void __launch_bounds__(kThreads) cg_vec_kernel(CGDev d, const T* __restrict__ kappa, T* __restrict__ out) {
  constexpr int NDP = NDOF + 1;
  constexpr int NPT = 4 * ((NQ + 3) / 4);
  extern __shared__ __align__(16) unsigned char smem[];
  T* s_tab = reinterpret_cast<T*>(smem);  // [NPT][4][NDP]
  T* s_slot = s_tab + NPT * 4 * NDP;
  const T* tab = static_cast<const T*>(d.tab);
  for (int i = threadIdx.x; i < NPT * 4 * NDP; i += kThreads) s_tab[i] = tab[i];
  const int ncp = d.ncp, nc = d.n_cell;
  const T* geo = static_cast<const T*>(d.geo);
  const T* qw = static_cast<const T*>(d.qw);
  const bool has_mass = d.sigma != 0.0;
  const T sigma = (T)d.sigma;
  int first, last, stride;
  xcd_range(d.n_blocks, first, last, stride);
  for (int b = first; b < last; b += stride) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kBlockCells * NDOF; idx += kThreads) {
      const int cl = idx % kBlockCells, j = idx / kBlockCells;
      const int cell = b * kBlockCells + cl;
      if (cell >= nc) continue;
      T acc = 0;
      for (int q = 0; q < NQ; ++q) {
        // geometry (c, q) of curved cells (16-cell tiles), or row c of
        // straight ones
        const long gr = CURV ? lanes::curved_geo_index(NQ, 0, q, cell) : (long)cell;
        const long gs = CURV ? (long)NQ * 16 : (long)ncp;
        const T G0 = geo[gr], G1 = geo[gs + gr], G2 = geo[2 * gs + gr];
        const T G3 = geo[3 * gs + gr], G4 = geo[4 * gs + gr], G5 = geo[5 * gs + gr];
        const T adet = geo[6 * gs + gr];
        const T w = qw[q];
        const T c = kappa ? kappa[lanes::cell_data_index(NQ, q, cell)] : T(1);
        const T x = s_tab[(q * 4 + 0) * NDP + j], y = s_tab[(q * 4 + 1) * NDP + j];
        const T z = s_tab[(q * 4 + 2) * NDP + j], val = s_tab[(q * 4 + 3) * NDP + j];
        if (MODE == MODE_DIAG) {
          acc += c * w * (G0 * x * x + G3 * y * y + G5 * z * z + T(2) * (G1 * x * y + G2 * x * z + G4 * y * z));
          if (has_mass) acc += sigma * w * adet * val * val;
        } else {
          acc += w * adet * c * val;
        }
      }
      s_slot[d.pos[j * ncp + cell]] = acc;
    }
    __syncthreads();
    cg_reduce<T>(d, s_slot, d.blk_nbd[b], d.blk_npriv[b], d.blk_priv_start[b], d.blk_other_off[b],
                 d.blk_ptr_off[b], out, static_cast<T*>(d.partials));
  }
}

// Shared DoFs: sum of the per-block partials in block order.  Constrained
// DoFs: identity rows (apply/backward), 1 (diagonal), 0 (load vector).
// blockIdx.y: the component of a vector field (partials, u and out offset by
// one component each).  Each thread takes kCombinePer entries i0, i0 + stride,
// ... and issues their loads together: the slot ranges, then the first four
// partial sums of each (at least two per shared DoF, checked at set-up).
constexpr int kCombinePer = 2;

template <typename T, int MODE>
__global__ void __launch_bounds__(256) cg_combine(CGDev d, const T* __restrict__ u, T* __restrict__ out) {
  const int stride = gridDim.x * 256;
  const int i0 = blockIdx.x * 256 + threadIdx.x;
  const long cofs = (long)blockIdx.y * d.n_dofs;
  const T* part = static_cast<const T*>(d.partials) + (long)blockIdx.y * d.n_partials;
  if (u) u += cofs;
  out += cofs;
  if (d.n_shared > 0) {
    // entries past the shared DoFs load the last one's range (in bounds) and
    // store nothing
    int p0[kCombinePer], p1[kCombinePer], gid[kCombinePer];
    T a[kCombinePer][4];
#pragma unroll
    for (int k = 0; k < kCombinePer; ++k) {
      const int i = min(i0 + k * stride, d.n_shared - 1);
      p0[k] = d.sh_ptr[i];
      p1[k] = d.sh_ptr[i + 1];
      gid[k] = d.sh_gid[i];
    }
#pragma unroll
    for (int k = 0; k < kCombinePer; ++k) {
      a[k][0] = part[p0[k]];
      a[k][1] = part[p0[k] + 1];
      a[k][2] = p0[k] + 2 < p1[k] ? part[p0[k] + 2] : T(0);
      a[k][3] = p0[k] + 3 < p1[k] ? part[p0[k] + 3] : T(0);
    }
#pragma unroll
    for (int k = 0; k < kCombinePer; ++k) {
      if (i0 + k * stride >= d.n_shared) continue;
      T s = 0;
      s += a[k][0];
      s += a[k][1];
      if (p0[k] + 2 < p1[k]) s += a[k][2];
      if (p0[k] + 3 < p1[k]) s += a[k][3];
      for (int p = p0[k] + 4; p < p1[k]; ++p) s += part[p];
      out[gid[k]] = s;
    }
  }
#pragma unroll
  for (int k = 0; k < kCombinePer; ++k) {
    const int c = i0 + k * stride - d.n_shared;
    if (c >= 0 && c < d.n_dofs - d.n_free) {
      const int gi = d.n_free + c;
      out[gi] = (MODE == MODE_APPLY || MODE == MODE_BACKWARD) ? u[gi] : (MODE == MODE_DIAG ? T(1) : T(0));
    }
  }
}

template <typename T, int MODE>
hipError_t launch_combine(const CGDev& d, const void* src, void* out, hipStream_t s, int ncomp = 1) {
  const int nfix = d.n_shared + (d.n_dofs - d.n_free);
  if (nfix > 0)
    hipLaunchKernelGGL((cg_combine<T, MODE>), dim3((nfix + 256 * kCombinePer - 1) / (256 * kCombinePer), ncomp),
                       dim3(256), 0, s, d, (const T*)src, (T*)out);
  return hipGetLastError();
}

template <typename T, int NDOF, int NQ, int C, int MODE, bool BF, bool CURV, int NCOMP>
hipError_t launch_cg_mf(const CGDev& d, const void* u, const void* g, const void* kappa, void* out, void* dk,
                        hipStream_t s, hipEvent_t* ev) {
  using TL = typename EngineSel<T, NDOF, NQ, C, BF>::type;
  const int ustage = (MODE == MODE_BACKWARD ? 2 : 1) * d.nbd_max;
  const size_t lds = (size_t)TL::LDS_BYTES + (size_t)(TL::NPT + kBlockCells * NDOF + ustage) * sizeof(T) +
                     (size_t)NDOF * kBlockCells * sizeof(uint16_t);
  if (lds > 160 * 1024) return hipErrorInvalidConfiguration;
  auto kern = cg_kernel<T, NDOF, NQ, C, MODE, BF, CURV, NCOMP>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = persistent_grid((const void*)kern, lds, d.n_blocks);
  // With ev: the start and end timestamps of this dispatch (no separate
  // marker packet, so back-to-back launches stay back to back).
  hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr, 0u, d,
                        (const T*)u, (const T*)g, (const T*)kappa, (T*)out, (T*)dk);
  e = hipGetLastError();
  if (e != hipSuccess || out == nullptr) return e;
  return launch_combine<T, MODE>(d, MODE == MODE_BACKWARD ? g : u, out, s, NCOMP);
}

template <typename T, int NDOF, int NQ, int MODE, bool CURV>
hipError_t launch_cg_vec(const CGDev& d, const void* kappa, void* out, hipStream_t s, hipEvent_t* ev) {
  constexpr int NPT = 4 * ((NQ + 3) / 4);
  const size_t lds = (size_t)(NPT * 4 * (NDOF + 1) + kBlockCells * NDOF) * sizeof(T);
  auto kern = cg_vec_kernel<T, NDOF, NQ, MODE, CURV>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = persistent_grid((const void*)kern, lds, d.n_blocks);
  hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr, 0u, d,
                        (const T*)kappa, (T*)out);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_combine<T, MODE>(d, nullptr, out, s);
}

template <typename T, int NDOF, int NQ, bool BF, bool CURV, int NCOMP>
hipError_t launch_cg_geo(const CGDev& d, int mode, const void* u, const void* g, const void* kappa, void* out,
                         void* dk, hipStream_t s, hipEvent_t* ev, bool* supported) {
  const bool mass = d.sigma != 0.0;
  switch (mode) {
    case MODE_APPLY:
      return mass ? launch_cg_mf<T, NDOF, NQ, 4, MODE_APPLY, BF, CURV, NCOMP>(d, u, g, kappa, out, dk, s, ev)
                  : launch_cg_mf<T, NDOF, NQ, 3, MODE_APPLY, BF, CURV, NCOMP>(d, u, g, kappa, out, dk, s, ev);
    case MODE_BACKWARD:
      if (BF) {
        *supported = false;
        return hipSuccess;
      }
      return mass ? launch_cg_mf<T, NDOF, NQ, 4, MODE_BACKWARD, false, CURV, NCOMP>(d, u, g, kappa, out, dk, s, ev)
                  : launch_cg_mf<T, NDOF, NQ, 3, MODE_BACKWARD, false, CURV, NCOMP>(d, u, g, kappa, out, dk, s, ev);
    // the diagonal and load vector are per component (tetmf.cpp replicates them)
    case MODE_DIAG: return launch_cg_vec<T, NDOF, NQ, MODE_DIAG, CURV>(d, kappa, out, s, ev);
    default: return launch_cg_vec<T, NDOF, NQ, MODE_LOAD, CURV>(d, kappa, out, s, ev);
  }
}

template <typename T, int NDOF, int NQ, bool BF, bool CURV>
hipError_t launch_cg_comp(const CGDev& d, int mode, const void* u, const void* g, const void* kappa, void* out,
                          void* dk, hipStream_t s, hipEvent_t* ev, bool* supported) {
  if (d.ncomp == 3 && (mode == MODE_APPLY || mode == MODE_BACKWARD)) {
    if constexpr (BF) {
      *supported = false;
      return hipSuccess;
    } else {
      return launch_cg_geo<T, NDOF, NQ, false, CURV, 3>(d, mode, u, g, kappa, out, dk, s, ev, supported);
    }
  }
  return launch_cg_geo<T, NDOF, NQ, BF, CURV, 1>(d, mode, u, g, kappa, out, dk, s, ev, supported);
}

template <typename T, int NDOF, int NQ, bool BF>
hipError_t launch_cg_mode(const CGDev& d, int mode, const void* u, const void* g, const void* kappa, void* out,
                          void* dk, hipStream_t s, hipEvent_t* ev, bool* supported) {
  return d.curved ? launch_cg_comp<T, NDOF, NQ, BF, true>(d, mode, u, g, kappa, out, dk, s, ev, supported)
                  : launch_cg_comp<T, NDOF, NQ, BF, false>(d, mode, u, g, kappa, out, dk, s, ev, supported);
}

template <typename T, bool BF>
hipError_t launch_cg_shape(const CGDev& d, int ndof, int nq, int mode, const void* u, const void* g,
                           const void* kappa, void* out, void* dk, hipStream_t s, bool* supported, hipEvent_t* ev) {
  *supported = true;
  if (ndof == 4 && nq == 4) return launch_cg_mode<T, 4, 4, BF>(d, mode, u, g, kappa, out, dk, s, ev, supported);
  if (ndof == 10 && nq == 4) return launch_cg_mode<T, 10, 4, BF>(d, mode, u, g, kappa, out, dk, s, ev, supported);
  if (ndof == 10 && nq == 14) return launch_cg_mode<T, 10, 14, BF>(d, mode, u, g, kappa, out, dk, s, ev, supported);
  if (ndof == 20 && nq == 14) return launch_cg_mode<T, 20, 14, BF>(d, mode, u, g, kappa, out, dk, s, ev, supported);
  if (ndof == 20 && nq == 24) return launch_cg_mode<T, 20, 24, BF>(d, mode, u, g, kappa, out, dk, s, ev, supported);
  *supported = false;
  return hipSuccess;
}

hipError_t launch_cg(const CGDev& d, int prec, int ndof, int nq, int mode, const void* u, const void* g,
                     const void* kappa, void* out, void* dk, hipStream_t s, bool* supported, hipEvent_t* ev) {
  if (prec == PREC_F64)
    return launch_cg_shape<double, false>(d, ndof, nq, mode, u, g, kappa, out, dk, s, supported, ev);
  if (prec == PREC_F32)
    return launch_cg_shape<float, false>(d, ndof, nq, mode, u, g, kappa, out, dk, s, supported, ev);
  return launch_cg_shape<float, true>(d, ndof, nq, mode, u, g, kappa, out, dk, s, supported, ev);
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

template <typename T, int NDOF, int NQ, int NQF, int C>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8)))
dg_kernel(DGDev d, const T* __restrict__ u, const T* __restrict__ kc, const T* __restrict__ kf, T* __restrict__ v) {
  using TC = Tile<T, NDOF, NQ, C>;
  using TF = Tile<T, NDOF, NQF, 4>;
  using M = Mfma<T>;
  typedef typename M::acc_t acc_t;
  extern __shared__ __align__(16) unsigned char smem[];
  T* s_tab = reinterpret_cast<T*>(smem);   // [NPT][C][NDP]
  T* s_ftab = s_tab + TC::TAB;              // [NPTF][4][NDP]
  T* s_qw = s_ftab + TF::TAB;
  T* s_fw = s_qw + TC::NPT;
  T* s_out = s_fw + TF::NPT;                // [kWaves][kTile * NDOF]
  int* s_perm = reinterpret_cast<int*>(s_out + kWaves * kTile * NDOF);
  {
    const T* tab = static_cast<const T*>(d.tab);
    for (int i = threadIdx.x; i < TC::TAB; i += kThreads) {
      const int col = i % TC::NDP, c = (i / TC::NDP) % C, p = i / (TC::NDP * C);
      s_tab[i] = (p < TC::NPT && col < NDOF) ? tab[(p * 4 + c) * TC::NDPG + col] : T(0);
    }
    const T* ftab = static_cast<const T*>(d.ftab);
    for (int i = threadIdx.x; i < TF::TAB; i += kThreads) {
      const int col = i % TF::NDP, c = (i / TF::NDP) % 4, p = i / (TF::NDP * 4);
      s_ftab[i] = (p < TF::NPT && col < NDOF) ? ftab[(p * 4 + c) * TF::NDPG + col] : T(0);
    }
    for (int i = threadIdx.x; i < TC::NPT; i += kThreads) s_qw[i] = static_cast<const T*>(d.qw)[i];
    for (int i = threadIdx.x; i < TF::NPT; i += kThreads) s_fw[i] = static_cast<const T*>(d.fw)[i];
    for (int i = threadIdx.x; i < 24 * NDOF; i += kThreads) s_perm[i] = d.perm[i];
  }
  __syncthreads();
  // the wave index is uniform in the wave: scalar registers for the tile loop
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ncp = d.ncp, nc = d.n_cell, nf = d.n_face;
  const T* geo = static_cast<const T*>(d.geo);
  const T* fgeo = static_cast<const T*>(d.fgeo);
  const T sigma = (T)d.sigma;
  // tiles of this wave: contiguous tile ranges per XCD
  const int ntiles = ncp / kTile;
  const int nx = 8, x = blockIdx.x % nx;
  const int per = (gridDim.x / nx) * kWaves;
  const int first = (int)((long long)ntiles * x / nx) + (blockIdx.x / nx) * kWaves + wave;
  const int last = (int)((long long)ntiles * (x + 1) / nx);
  for (int tile = first; tile < last; tile += per) {
    // lane coordinates re-derived per tile (not held across the tile loop)
    const int tid = phase_tid();
    const int lane = tid & 63;
    const int g = lane >> 4, c16 = lane & 15;
    T* so = s_out + (tid >> 6) * kTile * NDOF;
    const int cell0 = tile * kTile;
    const int cell = cell0 + c16;
    const bool valid = cell < nc;
    const int cc = valid ? cell : nc - 1;
    // ---- cell term
    {
      T ub[TC::KS];
      // the tile's DoF values from a uniform row base (cell0) and a 32-bit
      // lane offset below 16 NDOF sizeof(T), read at a valid cell and masked
      const T* ut = u + (long)cell0 * NDOF;
#pragma unroll
      for (int s = 0; s < TC::KS; ++s) {
        const int j = 4 * s + g;
        const T x = load_at(ut, (uint32_t)((cc - cell0) * NDOF + (j < NDOF ? j : NDOF - 1)) * (uint32_t)sizeof(T));
        ub[s] = (valid && j < NDOF) ? x : T(0);
      }
      // cell data: uniform row bases and 32-bit lane offsets (below 4 ncp
      // sizeof(T), within the set-up's 32-bit limit)
      const uint32_t coff = (uint32_t)cell * (uint32_t)sizeof(T);
      const T G0 = load_at(geo, coff), G1 = load_at(geo + (long)ncp, coff), G2 = load_at(geo + 2 * (long)ncp, coff);
      const T G3 = load_at(geo + 3 * (long)ncp, coff), G4 = load_at(geo + 4 * (long)ncp, coff);
      const T G5 = load_at(geo + 5 * (long)ncp, coff);
      const T adet = (C == 4) ? load_at(geo + 6 * (long)ncp, coff) : T(0);
      T kq[TC::KP];
      const T* kct = kc ? kc + lanes::cell_data_index(NQ, 0, cc & ~15) : nullptr;
#pragma unroll
      for (int k = 0; k < TC::KP; ++k)
        kq[k] = kc ? load_at(kct, (uint32_t)lanes::cell_data_index(NQ, 4 * k + lanes::kappa_lane_row(NQ, g, k), cc & 15) *
                                      (uint32_t)sizeof(T))
                   : T(1);
      acc_t acc[TC::MT];
      __builtin_amdgcn_s_setprio(1);  // matrix-core section at raised wave priority
      TC::interpolate(s_tab, ub, g, c16, acc);
#pragma unroll
      for (int k = 0; k < TC::KP; ++k) {
        const int q = g + 4 * k;
        const bool qok = valid && q < NQ;
        const T w = s_qw[q];
        const T s = qok ? kq[k] * w : T(0);
        const int i0 = C * k;
        const T xg = acc[i0 / 4][i0 % 4], yg = acc[(i0 + 1) / 4][(i0 + 1) % 4], zg = acc[(i0 + 2) / 4][(i0 + 2) % 4];
        T val = T(0);
        if constexpr (C == 4) val = acc[(i0 + 3) / 4][(i0 + 3) % 4];
        acc[i0 / 4][i0 % 4] = s * (G0 * xg + G1 * yg + G2 * zg);
        acc[(i0 + 1) / 4][(i0 + 1) % 4] = s * (G1 * xg + G3 * yg + G4 * zg);
        acc[(i0 + 2) / 4][(i0 + 2) % 4] = s * (G2 * xg + G4 * yg + G5 * zg);
        if constexpr (C == 4) acc[(i0 + 3) / 4][(i0 + 3) % 4] = qok ? sigma * w * adet * val : T(0);
      }
      acc_t vm;
      T vv[TC::NVA > 0 ? TC::NVA : 1];
      TC::integrate(s_tab, acc, g, c16, vm, vv);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (TC::NMF == 16 || M::row(g, r) < TC::NMF) so[c16 * NDOF + M::row(g, r)] = vm[r];
      if (TC::NVA > 0 && g < TC::NVA) {
        T mine = vv[0];
#pragma unroll
        for (int jj = 1; jj < (TC::NVA > 0 ? TC::NVA : 1); ++jj) mine = (g == jj) ? vv[jj] : mine;
        so[c16 * NDOF + 16 + g] = mine;
      }
      __builtin_amdgcn_s_setprio(0);
    }
    // ---- face terms.  Poisson form: each face's neighbour, relabelling code
    // and face id are requested one face ahead (115.1 -> 113.7 us at 32^3 x 6,
    // and no scratch); the mass-term form keeps those registers (it would
    // spill).
    constexpr bool kAhead = C == 3;
    int nbn = 0, coden = 0, fidn = 0;
    if constexpr (kAhead) {
      nbn = valid ? d.nb[cell] : -1;
      coden = valid ? d.code[cell] : 0;
      fidn = valid ? d.fid[cell] : 0;
    }
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      const long fi = (long)f * ncp + cell;
      int nbc, code, fidv;
      if constexpr (kAhead) {
        nbc = nbn;
        code = coden;
        fidv = fidn;
        if (f < 3) {
          nbn = valid ? d.nb[fi + ncp] : -1;
          coden = valid ? d.code[fi + ncp] : 0;
          fidn = valid ? d.fid[fi + ncp] : 0;
        }
      } else {
        nbc = valid ? d.nb[fi] : -1;
        code = valid ? d.code[fi] : 0;
        fidv = valid ? d.fid[fi] : 0;
      }
      const int ro = code & 255, rn = (code >> 8) & 255;
      const bool boundary = nbc < 0;
      const bool active = valid && (!boundary || d.dirichlet);
      T bo[3], bn[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        bo[q] = fgeo[((long)q * 4 + f) * ncp + cell];
        bn[q] = fgeo[((long)(3 + q) * 4 + f) * ncp + cell];
      }
      const T om = fgeo[((long)6 * 4 + f) * ncp + cell];
      const T tau = fgeo[((long)7 * 4 + f) * ncp + cell];
      T kfq[TF::KP];
#pragma unroll
      for (int k = 0; k < TF::KP; ++k) {
        const int q = g + 4 * k;
        kfq[k] = kf ? kf[(long)(q < NQF ? q : NQF - 1) * nf + fidv] : T(1);
      }
      T um[TF::KS], up[TF::KS];
      const int nbs = boundary ? cc : nbc;
#pragma unroll
      for (int s = 0; s < TF::KS; ++s) {
        const int j = 4 * s + g;
        const int jc = j < NDOF ? j : NDOF - 1;
        const T a = u[(long)cc * NDOF + s_perm[ro * NDOF + jc]];
        const T bq = u[(long)nbs * NDOF + s_perm[rn * NDOF + jc]];
        um[s] = (valid && j < NDOF) ? a : T(0);
        up[s] = (!boundary && j < NDOF) ? bq : T(0);
      }
      acc_t am[TF::MT], ap[TF::MT];
      __builtin_amdgcn_s_setprio(1);
      TF::interpolate(s_ftab, um, g, c16, am);
      TF::interpolate(s_ftab, up, g, c16, ap);
#pragma unroll
      for (int k = 0; k < TF::KP; ++k) {
        const int q = g + 4 * k;
        const bool qok = active && q < NQF;
        const T s = qok ? kfq[k] * s_fw[q] * om : T(0);
        const int i0 = 4 * k;
        const T dnm = bo[0] * am[i0 / 4][0] + bo[1] * am[i0 / 4][1] + bo[2] * am[i0 / 4][2];
        const T dnp = bn[0] * ap[i0 / 4][0] + bn[1] * ap[i0 / 4][1] + bn[2] * ap[i0 / 4][2];
        const T jump = boundary ? T(2) * am[i0 / 4][3] : am[i0 / 4][3] - ap[i0 / 4][3];
        const T avg = boundary ? dnm : T(0.5) * (dnm + dnp);
        const T cgr = T(-0.5) * s * jump;
        am[i0 / 4][0] = cgr * bo[0];
        am[i0 / 4][1] = cgr * bo[1];
        am[i0 / 4][2] = cgr * bo[2];
        am[i0 / 4][3] = s * (tau * jump - avg);
      }
      acc_t vf;
      T vvf[TF::NVA > 0 ? TF::NVA : 1];
      TF::integrate(s_ftab, am, g, c16, vf, vvf);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = M::row(g, r);
        if (TF::NMF == 16 || j < TF::NMF) so[c16 * NDOF + s_perm[ro * NDOF + j]] += vf[r];
      }
      if (TF::NVA > 0 && g < TF::NVA) {
        T mine = vvf[0];
#pragma unroll
        for (int jj = 1; jj < (TF::NVA > 0 ? TF::NVA : 1); ++jj) mine = (g == jj) ? vvf[jj] : mine;
        so[c16 * NDOF + s_perm[ro * NDOF + 16 + g]] += mine;
      }
      __builtin_amdgcn_s_setprio(0);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    // ---- store the tile (contiguous 16 x NDOF block of the DG vector)
    for (int i = lane; i < kTile * NDOF; i += 64)
      if (cell0 + i / NDOF < nc) v[(long)cell0 * NDOF + i] = so[i];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// Coefficient gradients of the SIPG operator, d(g^T A(kappa) u) / dkappa:
//   cell point q of cell e:   w_q (grad u . grad g)(x_q) |det J|
//   face point q of face F:   omega_q (-{{d_n g}} [[u]] - [[g]] {{d_n u}} + tau [[u]] [[g]])   (interior)
//                             omega_q (-g d_n u - u d_n g + 2 tau u g)                        (Dirichlet boundary)
//                             0                                                               (Neumann boundary)
// The bracket of an interior face is the same from either side; the side
// with the smaller library cell id writes it, so every face point is written
// once.  Traces are evaluated as in dg_kernel (common relabelled frame).
// Two interpolated fields are live at once in the cell term, so the register
// cap is relaxed to two waves per SIMD (no spills at P3 in FP64).
template <typename T, int NDOF, int NQ, int NQF>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 8)))
dg_grad_kernel(DGDev d, const T* __restrict__ u, const T* __restrict__ gv, T* __restrict__ dkc,
               T* __restrict__ dkf, int accumulate) {
  using TC = Tile<T, NDOF, NQ, 3>;
  using TF = Tile<T, NDOF, NQF, 4>;
  using M = Mfma<T>;
  typedef typename M::acc_t acc_t;
  extern __shared__ __align__(16) unsigned char smem[];
  T* s_tab = reinterpret_cast<T*>(smem);   // [NPTP][3][NDP]
  T* s_ftab = s_tab + TC::TAB;              // [NPTF][4][NDP]
  T* s_qw = s_ftab + TF::TAB;
  T* s_fw = s_qw + TC::NPT;
  int* s_perm = reinterpret_cast<int*>(s_fw + TF::NPT);
  {
    const T* tab = static_cast<const T*>(d.tab);
    for (int i = threadIdx.x; i < TC::TAB; i += kThreads) {
      const int col = i % TC::NDP, c = (i / TC::NDP) % 3, p = i / (TC::NDP * 3);
      s_tab[i] = (p < TC::NPT && col < NDOF) ? tab[(p * 4 + c) * TC::NDPG + col] : T(0);
    }
    const T* ftab = static_cast<const T*>(d.ftab);
    for (int i = threadIdx.x; i < TF::TAB; i += kThreads) {
      const int col = i % TF::NDP, c = (i / TF::NDP) % 4, p = i / (TF::NDP * 4);
      s_ftab[i] = (p < TF::NPT && col < NDOF) ? ftab[(p * 4 + c) * TF::NDPG + col] : T(0);
    }
    for (int i = threadIdx.x; i < TC::NPT; i += kThreads) s_qw[i] = static_cast<const T*>(d.qw)[i];
    for (int i = threadIdx.x; i < TF::NPT; i += kThreads) s_fw[i] = static_cast<const T*>(d.fw)[i];
    for (int i = threadIdx.x; i < 24 * NDOF; i += kThreads) s_perm[i] = d.perm[i];
  }
  __syncthreads();
  // the wave index is uniform in the wave: scalar registers for the tile loop
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ncp = d.ncp, nc = d.n_cell, nf = d.n_face;
  const T* geo = static_cast<const T*>(d.geo);
  const T* fgeo = static_cast<const T*>(d.fgeo);
  const int ntiles = ncp / kTile;
  const int nx = 8, x = blockIdx.x % nx;
  const int per = (gridDim.x / nx) * kWaves;
  const int first = (int)((long long)ntiles * x / nx) + (blockIdx.x / nx) * kWaves + wave;
  const int last = (int)((long long)ntiles * (x + 1) / nx);
  for (int tile = first; tile < last; tile += per) {
    const int tid = phase_tid();
    const int lane = tid & 63;
    const int g = lane >> 4, c16 = lane & 15;
    const int cell = tile * kTile + c16;
    const bool valid = cell < nc;
    const int cc = valid ? cell : nc - 1;
    if (dkc) {
      T ub[TC::KS], gb[TC::KS];
#pragma unroll
      for (int s = 0; s < TC::KS; ++s) {
        const int j = 4 * s + g;
        ub[s] = (valid && j < NDOF) ? u[(long)cell * NDOF + j] : T(0);
        gb[s] = (valid && j < NDOF) ? gv[(long)cell * NDOF + j] : T(0);
      }
      const T G0 = geo[0 * ncp + cell], G1 = geo[1 * ncp + cell], G2 = geo[2 * ncp + cell];
      const T G3 = geo[3 * ncp + cell], G4 = geo[4 * ncp + cell], G5 = geo[5 * ncp + cell];
      acc_t au[TC::MT], ag[TC::MT];
      TC::interpolate(s_tab, ub, g, c16, au);
      TC::interpolate(s_tab, gb, g, c16, ag);
#pragma unroll
      for (int k = 0; k < TC::KP; ++k) {
        const int q = g + 4 * k;
        const int i0 = 3 * k;
        const T ux = au[i0 / 4][i0 % 4], uy = au[(i0 + 1) / 4][(i0 + 1) % 4], uz = au[(i0 + 2) / 4][(i0 + 2) % 4];
        const T x_ = ag[i0 / 4][i0 % 4], y_ = ag[(i0 + 1) / 4][(i0 + 1) % 4], z_ = ag[(i0 + 2) / 4][(i0 + 2) % 4];
        const T val = s_qw[q] * (ux * (G0 * x_ + G1 * y_ + G2 * z_) + uy * (G1 * x_ + G3 * y_ + G4 * z_) +
                                 uz * (G2 * x_ + G4 * y_ + G5 * z_));
        if (valid && q < NQ) {
          const long di = lanes::cell_data_index(NQ, q, cell);
          dkc[di] = accumulate ? dkc[di] + val : val;
        }
      }
    }
    if (!dkf) continue;
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      const long fi = (long)f * ncp + cell;
      const int nbc = valid ? d.nb[fi] : -1;
      const int code = valid ? d.code[fi] : 0;
      const int fidv = valid ? d.fid[fi] : 0;
      const int ro = code & 255, rn = (code >> 8) & 255;
      const bool boundary = nbc < 0;
      // interior faces are written by the side with the smaller library cell id
      const bool writer = valid && (boundary || cell < nbc);
      T bo[3], bn[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        bo[q] = fgeo[((long)q * 4 + f) * ncp + cell];
        bn[q] = fgeo[((long)(3 + q) * 4 + f) * ncp + cell];
      }
      const T om = fgeo[((long)6 * 4 + f) * ncp + cell];
      const T tau = fgeo[((long)7 * 4 + f) * ncp + cell];
      const int nbs = boundary ? cc : nbc;
      // jump and average (own outward normal) of u, then of g, at the lane's points
      T ju[TF::KP], au_[TF::KP], jg[TF::KP], ag_[TF::KP];
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        const T* w = pass == 0 ? u : gv;
        T vm[TF::KS], vp[TF::KS];
#pragma unroll
        for (int s = 0; s < TF::KS; ++s) {
          const int j = 4 * s + g;
          const int jc = j < NDOF ? j : NDOF - 1;
          const T a = w[(long)cc * NDOF + s_perm[ro * NDOF + jc]];
          const T bq = w[(long)nbs * NDOF + s_perm[rn * NDOF + jc]];
          vm[s] = (valid && j < NDOF) ? a : T(0);
          vp[s] = (!boundary && j < NDOF) ? bq : T(0);
        }
        acc_t am[TF::MT], ap[TF::MT];
        TF::interpolate(s_ftab, vm, g, c16, am);
        TF::interpolate(s_ftab, vp, g, c16, ap);
#pragma unroll
        for (int k = 0; k < TF::KP; ++k) {
          const T dnm = bo[0] * am[k][0] + bo[1] * am[k][1] + bo[2] * am[k][2];
          const T dnp = bn[0] * ap[k][0] + bn[1] * ap[k][1] + bn[2] * ap[k][2];
          // boundary: the one-sided value and normal derivative
          const T jmp = boundary ? am[k][3] : am[k][3] - ap[k][3];
          const T avg = boundary ? dnm : T(0.5) * (dnm + dnp);
          if (pass == 0) {
            ju[k] = jmp;
            au_[k] = avg;
          } else {
            jg[k] = jmp;
            ag_[k] = avg;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < TF::KP; ++k) {
        const int q = g + 4 * k;
        const T omq = s_fw[q] * om;
        T val;
        if (boundary)
          val = d.dirichlet ? omq * (-jg[k] * au_[k] - ju[k] * ag_[k] + T(2) * tau * ju[k] * jg[k]) : T(0);
        else
          val = omq * (-ag_[k] * ju[k] - jg[k] * au_[k] + tau * ju[k] * jg[k]);
        if (writer && q < NQF) dkf[(long)q * nf + fidv] = accumulate ? dkf[(long)q * nf + fidv] + val : val;
      }
    }
  }
}

template <typename T, int NDOF, int NQ, int NQF, int C>
hipError_t launch_dg_t(const DGDev& d, const void* u, const void* kc, const void* kf, void* v, hipStream_t s,
                       hipEvent_t* ev) {
  using TC = Tile<T, NDOF, NQ, C>;
  using TF = Tile<T, NDOF, NQF, 4>;
  const size_t lds = (size_t)(TC::TAB + TF::TAB + TC::NPT + TF::NPT + kWaves * kTile * NDOF) * sizeof(T) +
                     24 * NDOF * sizeof(int);
  const int ntiles = d.ncp / kTile;
  auto kern = dg_kernel<T, NDOF, NQ, NQF, C>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = persistent_grid((const void*)kern, lds, (ntiles + kWaves - 1) / kWaves);
  hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, ev ? ev[0] : nullptr, ev ? ev[1] : nullptr, 0u, d,
                        (const T*)u, (const T*)kc, (const T*)kf, (T*)v);
  e = hipGetLastError();
  return e;
}

template <typename T>
hipError_t launch_dg_shape(const DGDev& d, int ndof, int nq, int nqf, const void* u, const void* kc, const void* kf,
                           void* v, hipStream_t s, bool* supported, hipEvent_t* ev) {
  *supported = true;
  const bool mass = d.sigma != 0.0;
#define TETMF_DG_CASE(ND, Q, QF)                                                         \
  if (ndof == ND && nq == Q && nqf == QF)                                                \
    return mass ? launch_dg_t<T, ND, Q, QF, 4>(d, u, kc, kf, v, s, ev)                   \
                : launch_dg_t<T, ND, Q, QF, 3>(d, u, kc, kf, v, s, ev);
  TETMF_DG_CASE(4, 4, 3)
  TETMF_DG_CASE(10, 14, 6)
  TETMF_DG_CASE(20, 24, 12)
#undef TETMF_DG_CASE
  *supported = false;
  return hipSuccess;
}

template <typename T, int NDOF, int NQ, int NQF>
hipError_t launch_dg_grad_t(const DGDev& d, const void* u, const void* g, void* dkc, void* dkf, bool acc,
                            hipStream_t s) {
  using TC = Tile<T, NDOF, NQ, 3>;
  using TF = Tile<T, NDOF, NQF, 4>;
  const size_t lds = (size_t)(TC::TAB + TF::TAB + TC::NPT + TF::NPT) * sizeof(T) + 24 * NDOF * sizeof(int);
  const int ntiles = d.ncp / kTile;
  auto kern = dg_grad_kernel<T, NDOF, NQ, NQF>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int grid = persistent_grid((const void*)kern, lds, (ntiles + kWaves - 1) / kWaves);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, s, d, (const T*)u, (const T*)g, (T*)dkc, (T*)dkf,
                     acc ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dg_grad_shape(const DGDev& d, int ndof, int nq, int nqf, const void* u, const void* g, void* dkc,
                                void* dkf, bool acc, hipStream_t s, bool* supported) {
  *supported = true;
  if (ndof == 4 && nq == 4 && nqf == 3) return launch_dg_grad_t<T, 4, 4, 3>(d, u, g, dkc, dkf, acc, s);
  if (ndof == 10 && nq == 14 && nqf == 6) return launch_dg_grad_t<T, 10, 14, 6>(d, u, g, dkc, dkf, acc, s);
  if (ndof == 20 && nq == 24 && nqf == 12) return launch_dg_grad_t<T, 20, 24, 12>(d, u, g, dkc, dkf, acc, s);
  *supported = false;
  return hipSuccess;
}

hipError_t launch_dg_grad(const DGDev& d, int prec, int ndof, int nq, int nqf, const void* u, const void* g,
                          void* dkc, void* dkf, bool accumulate, hipStream_t s, bool* supported) {
  if (prec == PREC_F64)
    return launch_dg_grad_shape<double>(d, ndof, nq, nqf, u, g, dkc, dkf, accumulate, s, supported);
  if (prec == PREC_F32)
    return launch_dg_grad_shape<float>(d, ndof, nq, nqf, u, g, dkc, dkf, accumulate, s, supported);
  *supported = false;
  return hipSuccess;
}

hipError_t launch_dg(const DGDev& d, int prec, int ndof, int nq, int nqf, const void* u, const void* kc,
                     const void* kf, void* v, hipStream_t s, bool* supported, hipEvent_t* ev) {
  if (prec == PREC_F64) return launch_dg_shape<double>(d, ndof, nq, nqf, u, kc, kf, v, s, supported, ev);
  if (prec == PREC_F32) return launch_dg_shape<float>(d, ndof, nq, nqf, u, kc, kf, v, s, supported, ev);
  *supported = false;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// layout of per-point cell data: user [n_cell][nq] FP64 <-> library [nq][n_cell]

// Per-point cell data between the user layout [n_cell][nq] (FP64, user cell
// order) and the library layout [nq][n_cell] (op precision, library order):
// a transpose with a gather/scatter over cells, staged through LDS so that
// both sides are read and written in whole rows (64 cells per workgroup;
// every user row of nq values is contiguous).
constexpr int kLayoutCells = 64;
static_assert(kLayoutCells % 16 == 0, "layout blocks hold whole 16-cell tiles");
constexpr int kLayoutMaxQ = 64;

template <typename T>
__global__ void __launch_bounds__(256) layout_kernel(int to_user, const int* __restrict__ perm, int nc, int nq,
                                                     const void* src, void* dst) {
  __shared__ double s[kLayoutCells * (kLayoutMaxQ + 1)];
  const int c0 = blockIdx.x * kLayoutCells;
  const int ncb = min(kLayoutCells, nc - c0);
  const int ld = nq + 1;  // odd row stride: the column reads hit distinct banks
  const int n = ncb * nq;
  // library side: the block's 16-cell tiles are one contiguous run of
  // nt 16 nq values (c0 is a multiple of 16); padding cells of the last tile
  // are written as zero
  const int nt = (ncb + 15) / 16;
  const long lbase = lanes::cell_data_index(nq, 0, c0);
  if (!to_user) {
    // user rows (coalesced within each row) -> LDS [cell][q]
    for (int i = threadIdx.x; i < n; i += 256) {
      const int cl = i / nq, q = i % nq;
      s[cl * ld + q] = static_cast<const double*>(src)[(long)perm[c0 + cl] * nq + q];
    }
    __syncthreads();
    // LDS -> library tiles [t][q][16]
    for (int i = threadIdx.x; i < nt * 16 * nq; i += 256) {
      const int t = i / (16 * nq), q = (i / 16) % nq, cl = 16 * t + i % 16;
      static_cast<T*>(dst)[lbase + i] = cl < ncb ? (T)s[cl * ld + q] : T(0);
    }
  } else {
    for (int i = threadIdx.x; i < nt * 16 * nq; i += 256) {
      const int t = i / (16 * nq), q = (i / 16) % nq, cl = 16 * t + i % 16;
      if (cl < ncb) s[cl * ld + q] = (double)static_cast<const T*>(src)[lbase + i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += 256) {
      const int cl = i / nq, q = i % nq;
      static_cast<double*>(dst)[(long)perm[c0 + cl] * nq + q] = s[cl * ld + q];
    }
  }
}

hipError_t launch_layout(int prec, int to_user, const int* cell_perm, int n_cell, int nq, const void* src, void* dst,
                         hipStream_t s) {
  if (nq < 1 || nq > kLayoutMaxQ || n_cell < 1) return hipErrorInvalidValue;
  const int grid = (n_cell + kLayoutCells - 1) / kLayoutCells;
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
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
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
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
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

// Fused Jacobi-PCG steps.  kVecBlocks blocks of 256 threads, grid-stride
// loops in a fixed order; every block writes one FP64 partial sum per dot
// product, and the consumers add the kVecBlocks partials in a fixed order
// (each consuming block computes the identical total), so all scalars are
// bitwise reproducible.
constexpr int kVecBlocks = 512;
// Elements per thread whose loads are issued together in the PCG vector
// kernels; each thread still visits its elements in increasing index order,
// so the per-thread sums are the same as with one element at a time.
constexpr int kVecUnroll = 4;

// Fixed-order sum over the block (256 threads) of v; the result in all threads.
__device__ inline double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Sum of the kVecBlocks partials (fixed order), in all threads.
__device__ inline double sum_partials(const double* __restrict__ part, double* sh) {
  double v = 0;
  for (int i = threadIdx.x; i < kVecBlocks; i += 256) v += part[i];
  return block_sum256(v, sh);
}

// x = 0, r = rhs, z = dinv r, p = z (unless keep_p); partials of r.z and r.r.
template <typename T>
__global__ void __launch_bounds__(256) pcg_init_kernel(const T* __restrict__ rhs, const T* __restrict__ dinv,
                                                       T* __restrict__ x, T* __restrict__ r, T* __restrict__ z,
                                                       T* __restrict__ p, double* __restrict__ part_rz,
                                                       double* __restrict__ part_rr, long n, int keep_p) {
  __shared__ double sh[256];
  double srz = 0, srr = 0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)kVecBlocks * 256) {
    const T ri = rhs[i], zi = dinv[i] * ri;
    x[i] = T(0);
    r[i] = ri;
    z[i] = zi;
    if (!keep_p) p[i] = zi;
    srz += (double)ri * (double)zi;
    srr += (double)ri * (double)ri;
  }
  srz = block_sum256(srz, sh);
  srr = block_sum256(srr, sh);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = srz;
    part_rr[blockIdx.x] = srr;
  }
}

// rz = sum(part_rz), rr = sum(part_rr) (one block).
__global__ void __launch_bounds__(256) pcg_scalars_kernel(const double* __restrict__ part_rz,
                                                          const double* __restrict__ part_rr, double* __restrict__ rz,
                                                          double* __restrict__ rr) {
  __shared__ double sh[256];
  const double a = sum_partials(part_rz, sh), b = sum_partials(part_rr, sh);
  if (threadIdx.x == 0) {
    *rz = a;
    *rr = b;
  }
}

// partials of p.q
template <typename T>
__global__ void __launch_bounds__(256) pcg_dot_kernel(const T* __restrict__ a, const T* __restrict__ b,
                                                      double* __restrict__ part, long n) {
  __shared__ double sh[256];
  constexpr long S = (long)kVecBlocks * 256;
  double v = 0;
  long i = (long)blockIdx.x * 256 + threadIdx.x;
  for (; i + (kVecUnroll - 1) * S < n; i += kVecUnroll * S) {
    T av[kVecUnroll], bv[kVecUnroll];
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      av[u] = a[i + u * S];
      bv[u] = b[i + u * S];
    }
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) v += (double)av[u] * (double)bv[u];
  }
  for (; i < n; i += S) v += (double)a[i] * (double)b[i];
  v = block_sum256(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// alpha = rz / p.q;  x += alpha p, r -= alpha q, z = dinv r;  partials of r.z, r.r
template <typename T>
__global__ void __launch_bounds__(256) pcg_xr_kernel(T* __restrict__ x, T* __restrict__ r, T* __restrict__ z,
                                                     const T* __restrict__ p, const T* __restrict__ q,
                                                     const T* __restrict__ dinv, const double* __restrict__ part_pq,
                                                     const double* __restrict__ rz, double* __restrict__ part_rz,
                                                     double* __restrict__ part_rr, double* __restrict__ pq_out,
                                                     long n) {
  __shared__ double sh[256];
  const double pq = sum_partials(part_pq, sh);
  if (pq_out && blockIdx.x == 0 && threadIdx.x == 0) *pq_out = pq;
  const T a = (T)(*rz / pq);
  constexpr long S = (long)kVecBlocks * 256;
  double srz = 0, srr = 0;
  long i = (long)blockIdx.x * 256 + threadIdx.x;
  for (; i + (kVecUnroll - 1) * S < n; i += kVecUnroll * S) {
    T xv[kVecUnroll], pv[kVecUnroll], rv[kVecUnroll], qv[kVecUnroll], dv[kVecUnroll];
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      const long k = i + u * S;
      xv[u] = x[k];
      pv[u] = p[k];
      rv[u] = r[k];
      qv[u] = q[k];
      dv[u] = dinv[k];
    }
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      const long k = i + u * S;
      x[k] = xv[u] + a * pv[u];
      const T ri = rv[u] - a * qv[u];
      const T zi = dv[u] * ri;
      r[k] = ri;
      z[k] = zi;
      srz += (double)ri * (double)zi;
      srr += (double)ri * (double)ri;
    }
  }
  for (; i < n; i += S) {
    x[i] += a * p[i];
    const T ri = r[i] - a * q[i];
    const T zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    srz += (double)ri * (double)zi;
    srr += (double)ri * (double)ri;
  }
  srz = block_sum256(srz, sh);
  srr = block_sum256(srr, sh);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = srz;
    part_rr[blockIdx.x] = srr;
  }
}

// rz_new = sum(part_rz), beta = rz_new / rz_old, p = z + beta p; block 0
// stores rz_new and rr (the scalars are double-buffered by the caller, so no
// block reads rz_old after it is replaced).
template <typename T>
__global__ void __launch_bounds__(256) pcg_p_kernel(T* __restrict__ p, const T* __restrict__ z,
                                                    const double* __restrict__ part_rz,
                                                    const double* __restrict__ part_rr,
                                                    const double* __restrict__ rz_old, double* __restrict__ rz_new,
                                                    double* __restrict__ rr, long n) {
  __shared__ double sh[256];
  const double rzn = sum_partials(part_rz, sh);
  const T beta = (T)(rzn / *rz_old);
  constexpr long S = (long)kVecBlocks * 256;
  long i = (long)blockIdx.x * 256 + threadIdx.x;
  for (; i + (kVecUnroll - 1) * S < n; i += kVecUnroll * S) {
    T zv[kVecUnroll], pv[kVecUnroll];
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) {
      zv[u] = z[i + u * S];
      pv[u] = p[i + u * S];
    }
#pragma unroll
    for (int u = 0; u < kVecUnroll; ++u) p[i + u * S] = zv[u] + beta * pv[u];
  }
  for (; i < n; i += S) p[i] = z[i] + beta * p[i];
  if (blockIdx.x == 0) {
    const double rrn = sum_partials(part_rr, sh);
    if (threadIdx.x == 0) {
      *rz_new = rzn;
      *rr = rrn;
    }
  }
}

// One Chebyshev-Jacobi step: r = b - (ax ? ax : 0), d = cd d + cr dinv r
// (d not read when cd_read is 0), x = (x_read ? x : 0) + d.
template <typename T>
__global__ void __launch_bounds__(256) cheb_step_kernel(const T* __restrict__ b, const T* __restrict__ ax,
                                                        const T* __restrict__ dinv, T* __restrict__ d,
                                                        T* __restrict__ x, T cd, T cr, int d_read, int x_read,
                                                        long n) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const T r = ax ? b[i] - ax[i] : b[i];
    const T di = (d_read ? cd * d[i] : T(0)) + cr * (dinv[i] * r);
    d[i] = di;
    x[i] = (x_read ? x[i] : T(0)) + di;
  }
}

// x_i in [-1, 1) from the SplitMix64 output function (Steele, Lea and Flood,
// 2014) applied to i: a reproducible start vector.
template <typename T>
__global__ void hash_fill_kernel(T* __restrict__ x, long n) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (T)((double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0);
  }
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

hipError_t pcg_init(int prec, const void* rhs, const void* dinv, void* x, void* r, void* z, void* p, double* part,
                    double* rz, double* rr, int64_t n, hipStream_t s, int keep_p) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(pcg_init_kernel<double>, dim3(kVecBlocks), dim3(256), 0, s, (const double*)rhs,
                       (const double*)dinv, (double*)x, (double*)r, (double*)z, (double*)p, part + kVecBlocks,
                       part + 2 * kVecBlocks, (long)n, keep_p);
  else
    hipLaunchKernelGGL(pcg_init_kernel<float>, dim3(kVecBlocks), dim3(256), 0, s, (const float*)rhs,
                       (const float*)dinv, (float*)x, (float*)r, (float*)z, (float*)p, part + kVecBlocks,
                       part + 2 * kVecBlocks, (long)n, keep_p);
  hipLaunchKernelGGL(pcg_scalars_kernel, dim3(1), dim3(256), 0, s, part + kVecBlocks, part + 2 * kVecBlocks, rz, rr);
  return hipGetLastError();
}

hipError_t pcg_iteration(int prec, void* x, void* r, void* z, void* p, const void* q, const void* dinv, double* part,
                         const double* rz_old, double* rz_new, double* rr, double* pq_out, int64_t n, hipStream_t s) {
  if (prec == PREC_F64) {
    hipLaunchKernelGGL(pcg_dot_kernel<double>, dim3(kVecBlocks), dim3(256), 0, s, (const double*)p, (const double*)q,
                       part, (long)n);
    hipLaunchKernelGGL(pcg_xr_kernel<double>, dim3(kVecBlocks), dim3(256), 0, s, (double*)x, (double*)r, (double*)z,
                       (const double*)p, (const double*)q, (const double*)dinv, part, rz_old, part + kVecBlocks,
                       part + 2 * kVecBlocks, pq_out, (long)n);
    hipLaunchKernelGGL(pcg_p_kernel<double>, dim3(kVecBlocks), dim3(256), 0, s, (double*)p, (const double*)z,
                       part + kVecBlocks, part + 2 * kVecBlocks, rz_old, rz_new, rr, (long)n);
  } else {
    hipLaunchKernelGGL(pcg_dot_kernel<float>, dim3(kVecBlocks), dim3(256), 0, s, (const float*)p, (const float*)q,
                       part, (long)n);
    hipLaunchKernelGGL(pcg_xr_kernel<float>, dim3(kVecBlocks), dim3(256), 0, s, (float*)x, (float*)r, (float*)z,
                       (const float*)p, (const float*)q, (const float*)dinv, part, rz_old, part + kVecBlocks,
                       part + 2 * kVecBlocks, pq_out, (long)n);
    hipLaunchKernelGGL(pcg_p_kernel<float>, dim3(kVecBlocks), dim3(256), 0, s, (float*)p, (const float*)z,
                       part + kVecBlocks, part + 2 * kVecBlocks, rz_old, rz_new, rr, (long)n);
  }
  return hipGetLastError();
}

hipError_t cheb_step(int prec, const void* b, const void* ax, const void* dinv, void* d, void* x, double cd,
                     double cr, int d_read, int x_read, int64_t n, hipStream_t s) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(cheb_step_kernel<double>, dim3(vgrid(n)), dim3(256), 0, s, (const double*)b, (const double*)ax,
                       (const double*)dinv, (double*)d, (double*)x, cd, cr, d_read, x_read, (long)n);
  else
    hipLaunchKernelGGL(cheb_step_kernel<float>, dim3(vgrid(n)), dim3(256), 0, s, (const float*)b, (const float*)ax,
                       (const float*)dinv, (float*)d, (float*)x, (float)cd, (float)cr, d_read, x_read, (long)n);
  return hipGetLastError();
}

hipError_t vec_hash_fill(int prec, void* x, int64_t n, hipStream_t s) {
  if (prec == PREC_F64)
    hipLaunchKernelGGL(hash_fill_kernel<double>, dim3(vgrid(n)), dim3(256), 0, s, (double*)x, (long)n);
  else
    hipLaunchKernelGGL(hash_fill_kernel<float>, dim3(vgrid(n)), dim3(256), 0, s, (float*)x, (long)n);
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

// ---------------------------------------------------------------------------
// Fixed device scratch of tetmf_apply_noalloc (callers that cannot allocate):
// the interface partial sums of a CG apply live in this array instead of the
// op's own buffer.  Every GPU the library runs on holds its own copy until
// the process ends.  In host code the array's name is only a host-side
// stand-in: noalloc_scratch() resolves the device address of the copy on the
// current device once (hipGetSymbolAddress) and every later use takes that
// address.  The partial sums need no clearing: the cell kernel writes every
// one of them before the combine kernel reads it.
static __device__ __align__(256) unsigned char scratch[TETMF_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace tetmf
