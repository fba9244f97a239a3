// Host side of the tetmf C ABI: mesh and operator setup, argument checking,
// dispatch to the HIP kernels, and the solver driver.
//
// Setup follows the data structures the paper describes for its matrix-free
// operator (Sec. 2.2-2.4): precomputed affine geometry per cell, one table of
// reference basis values and gradients at the quadrature points shared by all
// cells (eq. (6)), global DoF indices per cell (eq. (8)), face neighbour and
// face geometry data for the SIPG face terms (eq. (10)), and a locality
// preserving cell order (Sec. 2.5).  The GPU layout of each of them is
// described where it is built.
#include "../../include/tetmf.h"
#include "internal.h"
#include "lane_map.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

using namespace tetmf;

// ---------------------------------------------------------------------------
// errors

namespace {
thread_local std::string g_last_error;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

void check_hip(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) throw Error(TETMF_ERR_OUT_OF_MEMORY, std::string(what) + ": out of device memory");
  if (e != hipSuccess) throw Error(TETMF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(TETMF_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(TETMF_ERR_DEVICE, e.what());
  } catch (...) {
    return fail(TETMF_ERR_DEVICE, "unknown failure");
  }
}

// ---------------------------------------------------------------------------
// small dense helpers (host, setup only)

struct M3 {
  double a[3][3];
};

double det3(const M3& m) {
  return m.a[0][0] * (m.a[1][1] * m.a[2][2] - m.a[1][2] * m.a[2][1]) -
         m.a[0][1] * (m.a[1][0] * m.a[2][2] - m.a[1][2] * m.a[2][0]) +
         m.a[0][2] * (m.a[1][0] * m.a[2][1] - m.a[1][1] * m.a[2][0]);
}

M3 inv3(const M3& m) {
  double d = det3(m);
  M3 r;
  r.a[0][0] = (m.a[1][1] * m.a[2][2] - m.a[1][2] * m.a[2][1]) / d;
  r.a[0][1] = (m.a[0][2] * m.a[2][1] - m.a[0][1] * m.a[2][2]) / d;
  r.a[0][2] = (m.a[0][1] * m.a[1][2] - m.a[0][2] * m.a[1][1]) / d;
  r.a[1][0] = (m.a[1][2] * m.a[2][0] - m.a[1][0] * m.a[2][2]) / d;
  r.a[1][1] = (m.a[0][0] * m.a[2][2] - m.a[0][2] * m.a[2][0]) / d;
  r.a[1][2] = (m.a[0][2] * m.a[1][0] - m.a[0][0] * m.a[1][2]) / d;
  r.a[2][0] = (m.a[1][0] * m.a[2][1] - m.a[1][1] * m.a[2][0]) / d;
  r.a[2][1] = (m.a[0][1] * m.a[2][0] - m.a[0][0] * m.a[2][1]) / d;
  r.a[2][2] = (m.a[0][0] * m.a[1][1] - m.a[0][1] * m.a[1][0]) / d;
  return r;
}

// Jacobian with columns X1-X0, X2-X0, X3-X0 of the given vertex order.
M3 jacobian(const double* xyz, const int32_t* v) {
  M3 J;
  for (int k = 0; k < 3; ++k)
    for (int r = 0; r < 3; ++r) J.a[r][k] = xyz[3 * v[k + 1] + r] - xyz[3 * v[0] + r];
  return J;
}

// ---------------------------------------------------------------------------
// nodal basis: library node order and Vandermonde tabulation

// Library local node order ("entity order"): the 4 vertices, then the p-1
// nodes of each edge (0,1),(0,2),(0,3),(1,2),(1,3),(2,3) walking from the
// first vertex, then (p = 3) one node per face (0,1,2),(0,1,3),(0,2,3),(1,2,3).
// Node coordinates are sum_i alpha_i X_i / p.
std::vector<std::array<int, 4>> library_nodes(int p) {
  std::vector<std::array<int, 4>> out;
  for (int i = 0; i < 4; ++i) {
    std::array<int, 4> a{0, 0, 0, 0};
    a[i] = p;
    out.push_back(a);
  }
  const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (auto& e : E)
    for (int m = 1; m < p; ++m) {
      std::array<int, 4> a{0, 0, 0, 0};
      a[e[0]] = p - m;
      a[e[1]] = m;
      out.push_back(a);
    }
  if (p == 3) {
    const int F[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
    for (auto& f : F) {
      std::array<int, 4> a{0, 0, 0, 0};
      a[f[0]] = a[f[1]] = a[f[2]] = 1;
      out.push_back(a);
    }
  }
  return out;
}

// Monomial basis x^a y^b z^c, a+b+c <= p.
std::vector<std::array<int, 3>> monomials(int p) {
  std::vector<std::array<int, 3>> m;
  for (int a = 0; a <= p; ++a)
    for (int b = 0; a + b <= p; ++b)
      for (int c = 0; a + b + c <= p; ++c) m.push_back({a, b, c});
  return m;
}

long double ipow(long double x, int k) {
  long double r = 1;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

// Coefficients C (n x n) with phi_i(x) = sum_m C[m][i] mono_m(x), from the
// inverse of the Vandermonde matrix V[i][m] = mono_m(node_i).
std::vector<long double> vandermonde_inverse(int p) {
  auto nodes = library_nodes(p);
  auto mons = monomials(p);
  const int n = (int)nodes.size();
  std::vector<long double> V(n * n), C(n * n, 0);
  for (int i = 0; i < n; ++i) {
    long double x = (long double)nodes[i][1] / p, y = (long double)nodes[i][2] / p, z = (long double)nodes[i][3] / p;
    for (int m = 0; m < n; ++m) V[i * n + m] = ipow(x, mons[m][0]) * ipow(y, mons[m][1]) * ipow(z, mons[m][2]);
  }
  for (int i = 0; i < n; ++i) C[i * n + i] = 1;
  // Gauss-Jordan with partial pivoting on [V | I] -> [I | V^-1]
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs((double)V[r * n + col]) > std::fabs((double)V[piv * n + col])) piv = r;
    for (int k = 0; k < n; ++k) {
      std::swap(V[col * n + k], V[piv * n + k]);
      std::swap(C[col * n + k], C[piv * n + k]);
    }
    long double d = V[col * n + col];
    for (int k = 0; k < n; ++k) {
      V[col * n + k] /= d;
      C[col * n + k] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      long double f = V[r * n + col];
      if (f == 0) continue;
      for (int k = 0; k < n; ++k) {
        V[r * n + k] -= f * V[col * n + k];
        C[r * n + k] -= f * C[col * n + k];
      }
    }
  }
  // C now holds V^-1: phi_i = sum_m Vinv[m][i] mono_m
  return C;
}

// Reference values and gradients of the library basis at points x (n_pts x 3):
// out[(q * 4 + comp) * ndof + j], comp 0..2 = d/dx, d/dy, d/dz, comp 3 = value.
std::vector<double> tabulate(int p, const std::vector<double>& pts) {
  auto mons = monomials(p);
  const int n = (int)mons.size();
  auto C = vandermonde_inverse(p);
  const int np = (int)pts.size() / 3;
  std::vector<double> out((size_t)np * 4 * n, 0.0);
  for (int q = 0; q < np; ++q) {
    long double x = pts[3 * q], y = pts[3 * q + 1], z = pts[3 * q + 2];
    for (int m = 0; m < n; ++m) {
      int a = mons[m][0], b = mons[m][1], c = mons[m][2];
      long double val = ipow(x, a) * ipow(y, b) * ipow(z, c);
      long double dx = a ? a * ipow(x, a - 1) * ipow(y, b) * ipow(z, c) : 0;
      long double dy = b ? b * ipow(x, a) * ipow(y, b - 1) * ipow(z, c) : 0;
      long double dz = c ? c * ipow(x, a) * ipow(y, b) * ipow(z, c - 1) : 0;
      for (int j = 0; j < n; ++j) {
        long double cm = C[m * n + j];
        out[((size_t)q * 4 + 0) * n + j] += (double)0 + (double)(cm * dx);
        out[((size_t)q * 4 + 1) * n + j] += (double)(cm * dy);
        out[((size_t)q * 4 + 2) * n + j] += (double)(cm * dz);
        out[((size_t)q * 4 + 3) * n + j] += (double)(cm * val);
      }
    }
  }
  return out;
}

int mt_for(int n) { return (n + 3) / 4; }

}  // namespace

// ---------------------------------------------------------------------------
// mesh

struct tetmf_mesh {
  int64_t nv = 0, nc = 0, nf = 0, nif = 0;
  std::vector<double> xyz;
  std::vector<int32_t> tets;
  std::vector<int32_t> ftri;       // [nf][3] sorted vertex ids
  std::vector<int32_t> fcell;      // [nf][2] user cells (second -1 on the boundary), first < second
  std::vector<int8_t> flocal;      // [nf][2] local face index (= opposite vertex) in each cell
  std::vector<int32_t> cell_face;  // [nc][4] face id of local face f
  std::vector<double> vol;         // [nc] |det J| / 6
};

extern "C" int tetmf_mesh_create(int64_t n_vert, const double* xyz, int64_t n_cell, const int32_t* tets,
                                 tetmf_mesh** out) {
  return guarded([&]() -> int {
    if (!out || !xyz || !tets || n_vert < 4 || n_cell < 1 || n_cell > (int64_t)INT32_MAX / 4 ||
        n_vert > INT32_MAX)
      return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_mesh_create: invalid sizes or NULL pointers");
    *out = nullptr;
    auto m = new tetmf_mesh();
    std::unique_ptr<tetmf_mesh> guard(m);
    m->nv = n_vert;
    m->nc = n_cell;
    m->xyz.assign(xyz, xyz + 3 * n_vert);
    m->tets.assign(tets, tets + 4 * n_cell);
    for (int64_t i = 0; i < 4 * n_cell; ++i)
      if (m->tets[i] < 0 || m->tets[i] >= n_vert)
        return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_mesh_create: vertex id out of range in cell " +
                                                    std::to_string(i / 4));
    for (int64_t i = 0; i < 3 * n_vert; ++i)
      if (!std::isfinite(m->xyz[i])) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_mesh_create: non-finite coordinate");
    // degenerate / duplicated vertices
    double edge_sum = 0;
    m->vol.resize(n_cell);
    for (int64_t e = 0; e < n_cell; ++e) {
      const int32_t* v = &m->tets[4 * e];
      for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) {
          if (v[a] == v[b])
            return fail(TETMF_ERR_DEGENERATE_CELL, "tetmf_mesh_create: repeated vertex in cell " + std::to_string(e));
          double d2 = 0;
          for (int r = 0; r < 3; ++r) {
            double d = m->xyz[3 * v[a] + r] - m->xyz[3 * v[b] + r];
            d2 += d * d;
          }
          edge_sum += std::sqrt(d2);
        }
      m->vol[e] = std::fabs(det3(jacobian(m->xyz.data(), v))) / 6.0;
    }
    double h = edge_sum / (6.0 * n_cell);
    for (int64_t e = 0; e < n_cell; ++e)
      if (6.0 * m->vol[e] <= 1e-12 * h * h * h)
        return fail(TETMF_ERR_DEGENERATE_CELL, "tetmf_mesh_create: degenerate cell " + std::to_string(e));
    // faces: sorted triples, grouped
    struct FK {
      int32_t a, b, c;
      int32_t cf;  // cell * 4 + local face
    };
    std::vector<FK> fk((size_t)4 * n_cell);
    for (int64_t e = 0; e < n_cell; ++e) {
      const int32_t* v = &m->tets[4 * e];
      for (int f = 0; f < 4; ++f) {
        int32_t t[3];
        int k = 0;
        for (int i = 0; i < 4; ++i)
          if (i != f) t[k++] = v[i];
        std::sort(t, t + 3);
        fk[4 * e + f] = {t[0], t[1], t[2], (int32_t)(4 * e + f)};
      }
    }
    std::sort(fk.begin(), fk.end(), [](const FK& x, const FK& y) {
      if (x.a != y.a) return x.a < y.a;
      if (x.b != y.b) return x.b < y.b;
      if (x.c != y.c) return x.c < y.c;
      return x.cf < y.cf;
    });
    m->cell_face.assign((size_t)4 * n_cell, -1);
    size_t i = 0;
    while (i < fk.size()) {
      size_t j = i + 1;
      while (j < fk.size() && fk[j].a == fk[i].a && fk[j].b == fk[i].b && fk[j].c == fk[i].c) ++j;
      if (j - i > 2)
        return fail(TETMF_ERR_NONCONFORMING_MESH, "tetmf_mesh_create: a triangle is shared by more than two cells");
      int32_t fid = (int32_t)m->ftri.size() / 3;
      m->ftri.insert(m->ftri.end(), {fk[i].a, fk[i].b, fk[i].c});
      m->fcell.push_back(fk[i].cf / 4);
      m->flocal.push_back((int8_t)(fk[i].cf % 4));
      m->cell_face[fk[i].cf] = fid;
      if (j - i == 2) {
        m->fcell.push_back(fk[i + 1].cf / 4);
        m->flocal.push_back((int8_t)(fk[i + 1].cf % 4));
        m->cell_face[fk[i + 1].cf] = fid;
        m->nif++;
      } else {
        m->fcell.push_back(-1);
        m->flocal.push_back(-1);
      }
      i = j;
    }
    m->nf = (int64_t)m->ftri.size() / 3;
    *out = guard.release();
    return TETMF_OK;
  });
}

extern "C" void tetmf_mesh_destroy(tetmf_mesh* mesh) { delete mesh; }

extern "C" int tetmf_mesh_faces(const tetmf_mesh* mesh, int64_t* n_face, int64_t* n_interior) {
  if (!mesh) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_mesh_faces: NULL mesh");
  if (n_face) *n_face = mesh->nf;
  if (n_interior) *n_interior = mesh->nif;
  return TETMF_OK;
}

// ---------------------------------------------------------------------------
// operator

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct tetmf_op {
  int kind, degree, bc, prec, device;
  int ndof, nq, nqf, mt, mtf;
  int64_t nc, ncp, nf, nif, n_dofs, n_free, n_blocks = 0, n_shared = 0, n_partials = 0;
  double sigma, eta;
  std::vector<int32_t> cell_perm;  // library cell -> user cell
  std::vector<int32_t> user_to_lib;
  std::vector<double> dof_xyz;
  std::vector<int32_t> dof_cell;
  std::vector<DevBuf> bufs;
  int32_t* d_cell_perm = nullptr;
  CGDev cg{};
  DGDev dg{};
  double flops = 0, bytes = 0;          // algorithmic work of one apply
  double flops_bwd = 0, bytes_bwd = 0;  // and of one full backward
  int ncomp = 1;                 // components of a vector field (CG), stored one after another
  bool curved = false;
  const double* qjac = nullptr;  // per-point Jacobians during set-up only (user memory)
  const tetmf_mesh* mesh_tag = nullptr;
  int64_t mesh_nc = 0, mesh_nv = 0;
  // solver scratch (allocated on first solve) and smoother scratch (first smoothing)
  std::vector<DevBuf> solve_bufs;
  std::vector<DevBuf> cheb_bufs;
  // kernel timing (tetmf_op_profile)
  bool profiling = false;
  std::vector<hipEvent_t> events;  // pairs
  size_t events_used = 0;          // pairs recorded

  int64_t nvec() const { return n_dofs * ncomp; }  // length of the operator's vectors

  hipEvent_t* next_events() {
    if (!profiling) return nullptr;
    if (2 * events_used + 2 > events.size()) {
      hipEvent_t a, b;
      check_hip(hipEventCreate(&a), "hipEventCreate");
      check_hip(hipEventCreate(&b), "hipEventCreate");
      events.push_back(a);
      events.push_back(b);
    }
    return &events[2 * events_used++];
  }

  ~tetmf_op() {
    if (bufs.empty() && solve_bufs.empty() && cheb_bufs.empty() && events.empty()) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    for (auto& b : bufs) (void)hipFree(b.p);
    for (auto& b : solve_bufs) (void)hipFree(b.p);
    for (auto& b : cheb_bufs) (void)hipFree(b.p);
    for (auto e : events) (void)hipEventDestroy(e);
    (void)hipSetDevice(cur);
  }

  template <typename V>
  void* upload(const std::vector<V>& h) {
    size_t bytes = std::max<size_t>(h.size() * sizeof(V), 16);
    void* p = nullptr;
    check_hip(hipMalloc(&p, bytes), "hipMalloc");
    bufs.push_back({p, bytes});
    if (!h.empty()) check_hip(hipMemcpy(p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice), "hipMemcpy");
    return p;
  }
  void* alloc(size_t bytes) {
    void* p = nullptr;
    check_hip(hipMalloc(&p, std::max<size_t>(bytes, 16)), "hipMalloc");
    bufs.push_back({p, bytes});
    return p;
  }
  int64_t device_bytes() const {
    int64_t s = 0;
    for (auto& b : bufs) s += (int64_t)b.bytes;
    return s;
  }
  size_t esize() const { return prec == TETMF_F64 ? 8 : 4; }
  // upload a double array in the op's storage precision
  void* upload_real(const std::vector<double>& h) {
    if (prec == TETMF_F64) return upload(h);
    std::vector<float> f(h.begin(), h.end());
    return upload(f);
  }
};

namespace {

// Morton (Z-order) key of a point in the unit box, 21 bits per axis.
uint64_t spread21(uint64_t x) {
  x &= 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffULL;
  x = (x | x << 16) & 0x1f0000ff0000ffULL;
  x = (x | x << 8) & 0x100f00f00f00f00fULL;
  x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
  x = (x | x << 2) & 0x1249249249249249ULL;
  return x;
}

// Locality order of the cells (Sec. 2.5 motivates it; the method here is a
// space-filling curve rather than the paper's greedy grouping): sort by the
// Morton key of the centroid, ties by user id.
// Every per-lane read of the CG cell kernel instantiation that serves an
// operator, enumerated from the index maps the kernel itself uses
// (lane_map.h): each row inside its array, the split of a slot row into the
// uniform row base and the lane part that the kernel's loads rely on, and
// every 32-bit byte offset below 2^32 at ncp_max cells, the largest count the
// set-up accepts at this degree.  Throws DEVICE naming the failing map.
void check_lane_maps(int esize, int nd, int nq, int64_t ncp_max) {
  auto bad = [&](const std::string& what) {
    throw Error(TETMF_ERR_DEVICE, "kernel lane map (n_dof_cell " + std::to_string(nd) + ", n_q " +
                                      std::to_string(nq) + "): " + what);
  };
  const uint64_t lim = (uint64_t)1 << 32, n = (uint64_t)ncp_max;
  for (int g = 0; g < 4; ++g) {
    for (int r = 0; r < 4; ++r) {
      const int pr = lanes::pos_row(esize, nd, g, r);
      if (pr < -1 || pr >= nd) bad("slot-position row " + std::to_string(pr) + " outside the cell's DoFs");
      if (pr >= 0 && lanes::acc_row(esize, g, 0) + lanes::acc_row(esize, 0, r) != pr)
        bad("slot-position row is not row base + lane part");
      if (pr >= 0 && ((uint64_t)lanes::acc_row(esize, g, 0) * n + n - 1) * 2 >= lim)
        bad("slot-position offset beyond 32 bits");
    }
    const int tr = lanes::pos_tail_row(nd, g);
    if (lanes::n_tail(nd) > 0) {
      if (tr < 16 || tr >= nd) bad("tail slot-position row outside the cell's DoFs");
      if (((uint64_t)(tr - 16) * n + n - 1) * 2 >= lim) bad("tail slot-position offset beyond 32 bits");
    } else if (tr != -1) {
      bad("tail slot-position row without tail DoFs");
    }
    for (int k = 0; k < (nq + 3) / 4; ++k) {
      const int lr = lanes::kappa_lane_row(nq, g, k);
      if (lr < 0 || lr > 3 || 4 * k + lr >= nq) bad("coefficient row outside the rule");
      // offset inside the cell's 16-cell tile of the per-point data
      const long ci = lanes::cell_data_index(nq, 4 * k + lr, 15);
      if (ci < 0 || ci >= 16L * nq || (uint64_t)ci * esize >= lim) bad("coefficient offset outside its tile");
    }
  }
  for (int j = 0; j < 32; ++j) {
    const int o = lanes::operand_row(nd, j);
    if (o < 0 || o >= nd) bad("operand row outside the cell's DoFs");
  }
  // geometry (cell * size; curved: an offset inside a 16-cell tile) and
  // the block-index staging (2 (j ncp + cell in block))
  if ((4 * n - 1) * esize >= lim) bad("geometry offset beyond 32 bits");
  if (2 * ((uint64_t)(nd - 1) * n + 255) >= lim) bad("index staging offset beyond 32 bits");
}

std::vector<int32_t> locality_order(const tetmf_mesh& m) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < m.nv; ++v)
    for (int r = 0; r < 3; ++r) {
      lo[r] = std::min(lo[r], m.xyz[3 * v + r]);
      hi[r] = std::max(hi[r], m.xyz[3 * v + r]);
    }
  double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
  std::vector<std::pair<uint64_t, int32_t>> key(m.nc);
  for (int64_t e = 0; e < m.nc; ++e) {
    uint64_t code = 0;
    for (int r = 0; r < 3; ++r) {
      double c = 0;
      for (int i = 0; i < 4; ++i) c += m.xyz[3 * m.tets[4 * e + i] + r];
      c = (c / 4 - lo[r]) / ext;
      uint64_t q = (uint64_t)std::min(std::max(c * 2097151.0, 0.0), 2097151.0);
      code |= spread21(q) << r;
    }
    key[e] = {code, (int32_t)e};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> perm(m.nc);
  for (int64_t i = 0; i < m.nc; ++i) perm[i] = key[i].second;
  return perm;
}

// All 24 relabellings of the 4 vertices in lexicographic order.
std::vector<std::array<int, 4>> all_relabellings() {
  std::vector<std::array<int, 4>> out;
  std::array<int, 4> a{0, 1, 2, 3};
  do out.push_back(a);
  while (std::next_permutation(a.begin(), a.end()));
  return out;
}

int relabelling_id(const std::array<int, 4>& s) {
  static const auto all = all_relabellings();
  for (size_t i = 0; i < all.size(); ++i)
    if (all[i] == s) return (int)i;
  return -1;
}

void fill_tables(tetmf_op* op, const tetmf_op_desc* d) {
  // Cell table: rows (q, comp) for q < 4*MT (zero beyond n_q), row stride
  // ndof + 1 (odd, so that 16 lanes reading one column hit distinct LDS banks).
  const int p = op->degree, nd = op->ndof, ndp = nd + 1;
  std::vector<double> pts(d->q_points, d->q_points + 3 * op->nq);
  auto t = tabulate(p, pts);
  std::vector<double> tab((size_t)op->mt * 16 * ndp, 0.0), qw((size_t)op->mt * 4, 0.0);
  for (int q = 0; q < op->nq; ++q) {
    qw[q] = d->q_weights[q];
    for (int c = 0; c < 4; ++c)
      for (int j = 0; j < nd; ++j) tab[((size_t)q * 4 + c) * ndp + j] = t[((size_t)q * 4 + c) * nd + j];
  }
  const void* dtab = op->upload_real(tab);
  const void* dqw = op->upload_real(qw);
  if (op->kind == TETMF_CG) {
    op->cg.tab = dtab;
    op->cg.qw = dqw;
  } else {
    op->dg.tab = dtab;
    op->dg.qw = dqw;
    std::vector<double> fp((size_t)3 * op->nqf);
    for (int q = 0; q < op->nqf; ++q) {
      fp[3 * q] = d->qf_points[2 * q];
      fp[3 * q + 1] = d->qf_points[2 * q + 1];
      fp[3 * q + 2] = 0.0;
    }
    auto ft = tabulate(p, fp);
    std::vector<double> ftab((size_t)op->mtf * 16 * ndp, 0.0), fw((size_t)op->mtf * 4, 0.0);
    for (int q = 0; q < op->nqf; ++q) {
      fw[q] = d->qf_weights[q];
      for (int c = 0; c < 4; ++c)
        for (int j = 0; j < nd; ++j) ftab[((size_t)q * 4 + c) * ndp + j] = ft[((size_t)q * 4 + c) * nd + j];
    }
    op->dg.ftab = op->upload_real(ftab);
    op->dg.fw = op->upload_real(fw);
  }
}

// Per-cell geometry [7][ncp]: the six entries of G = |det J| J^-1 J^-T and |det J|.
std::vector<double> cell_geometry(const tetmf_mesh& m, const std::vector<int32_t>& perm, int64_t ncp) {
  std::vector<double> geo((size_t)7 * ncp, 0.0);
  for (int64_t i = 0; i < (int64_t)perm.size(); ++i) {
    const int32_t* v = &m.tets[4 * (int64_t)perm[i]];
    M3 J = jacobian(m.xyz.data(), v);
    double adet = std::fabs(det3(J));
    M3 Ji = inv3(J);
    double G[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += Ji.a[a][k] * Ji.a[b][k];
        G[a][b] = adet * s;
      }
    const double vals[7] = {G[0][0], G[0][1], G[0][2], G[1][1], G[1][2], G[2][2], adet};
    for (int k = 0; k < 7; ++k) geo[(size_t)k * ncp + i] = vals[k];
  }
  return geo;
}

// Per-point geometry of curved cells, in 16-cell tiles [ncp / 16][7][nq][16]
// (lanes::curved_geo_index): G_q = |det J_q| J_q^-1 J_q^-T and |det J_q| for
// each library cell and rule point, from the user's Jacobians
// [n_cell][nq][3][3] (user cell order); padding cells hold zeros.
std::vector<double> point_geometry(const double* jac, const std::vector<int32_t>& perm, int nq, int64_t ncp) {
  std::vector<double> geo((size_t)7 * nq * ncp, 0.0);
  for (int64_t i = 0; i < (int64_t)perm.size(); ++i)
    for (int q = 0; q < nq; ++q) {
      const double* a = &jac[((size_t)perm[i] * nq + q) * 9];
      M3 J;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J.a[r][c] = a[3 * r + c];
      const double adet = std::fabs(det3(J));
      M3 Ji = inv3(J);
      double G[3][3];
      for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) {
          double sum = 0;
          for (int k = 0; k < 3; ++k) sum += Ji.a[x][k] * Ji.a[y][k];
          G[x][y] = adet * sum;
        }
      const double vals[7] = {G[0][0], G[0][1], G[0][2], G[1][1], G[1][2], G[2][2], adet};
      for (int k = 0; k < 7; ++k) geo[(size_t)lanes::curved_geo_index(nq, k, q, i)] = vals[k];
    }
  return geo;
}

// Host invariants of the CG block data that the kernels rely on for every
// memory access (bounds of all indices, each (cell, node) slot used exactly
// once, CSR ranges monotone).  Empty string when everything holds.
std::string validate_cg(const tetmf_op* op, int nd, const std::vector<int32_t>& priv_start,
                        const std::vector<int32_t>& npriv, const std::vector<int32_t>& blk_nbd,
                        const std::vector<int32_t>& blk_other_off, const std::vector<int32_t>& blk_ptr_off,
                        const std::vector<int32_t>& other_gid, const std::vector<int32_t>& other_pslot,
                        const std::vector<uint16_t>& lidx, const std::vector<uint16_t>& pos,
                        const std::vector<uint16_t>& slot_ptr, const std::vector<int32_t>& sh_gid,
                        const std::vector<int32_t>& sh_ptr, int nbd_max) {
  const int64_t nb = op->n_blocks, nc = op->nc, ncp = op->ncp;
  auto bad = [](const std::string& s) { return "block data: " + s; };
  if ((int64_t)lidx.size() != nd * ncp || (int64_t)pos.size() != nd * ncp) return bad("lidx/pos size");
  if (other_gid.empty() || other_gid.size() != other_pslot.size()) return bad("other lists");
  if (sh_ptr.size() != sh_gid.size() + 1 || sh_ptr.back() != op->n_partials) return bad("shared CSR");
  // every shared DoF has at least two partial sums (cg_combine reads two unconditionally)
  for (size_t s = 0; s + 1 < sh_ptr.size(); ++s)
    if (sh_ptr[s] + 2 > sh_ptr[s + 1] || sh_gid[s] < 0 || sh_gid[s] >= op->n_free) return bad("shared entry");
  std::vector<int64_t> pslot_seen(op->n_partials, 0);
  std::vector<int64_t> owner(op->n_dofs, 0);
  for (int64_t b = 0; b < nb; ++b) {
    const int nbd = blk_nbd[b], np = npriv[b], ps = priv_start[b];
    if (nbd < np || nbd > nbd_max || nbd > kBlockCells * nd) return bad("nbd of block " + std::to_string(b));
    if (ps < 0 || ps + np > op->n_free) return bad("private range of block " + std::to_string(b));
    for (int k = 0; k < np; ++k) owner[ps + k]++;
    const int64_t oo = blk_other_off[b], po = blk_ptr_off[b];
    if (oo < 0 || oo + (nbd - np) > (int64_t)other_gid.size()) return bad("other offset of block " + std::to_string(b));
    if (po < 0 || po + nbd + 1 > (int64_t)slot_ptr.size()) return bad("slot_ptr offset of block " + std::to_string(b));
    for (int k = 0; k < nbd - np; ++k) {
      const int g = other_gid[oo + k], s = other_pslot[oo + k];
      if (g < 0 || g >= op->n_dofs) return bad("other gid");
      if ((g < op->n_free) != (s >= 0)) return bad("partial slot of a free/constrained DoF");
      if (s >= op->n_partials) return bad("partial slot range");
      if (s >= 0) pslot_seen[s]++;
    }
    const int c0 = (int)(b * kBlockCells), c1 = (int)std::min<int64_t>(nc, c0 + kBlockCells);
    const int nslot = (c1 - c0) * nd;
    if (slot_ptr[po] != 0 || slot_ptr[po + nbd] != nslot) return bad("slot ranges of block " + std::to_string(b));
    for (int k = 0; k < nbd; ++k)
      if (slot_ptr[po + k] > slot_ptr[po + k + 1]) return bad("slot ranges not monotone");
    std::vector<int> used(nslot, 0);
    for (int i = c0; i < c1; ++i)
      for (int j = 0; j < nd; ++j) {
        const int l = lidx[(size_t)j * ncp + i], q = pos[(size_t)j * ncp + i];
        if (l >= nbd) return bad("local index out of range");
        if (q < slot_ptr[po + l] || q >= slot_ptr[po + l + 1]) return bad("slot outside its DoF's range");
        used[q]++;
      }
    for (int q = 0; q < nslot; ++q)
      if (used[q] != 1) return bad("slot not used exactly once");
  }
  for (int64_t s = 0; s < op->n_partials; ++s)
    if (pslot_seen[s] != 1) return bad("partial slot not written exactly once");
  for (int64_t g = 0; g < op->n_free; ++g)
    if (owner[g] > 1) return bad("private DoF in two blocks");
  return "";
}

void setup_cg(tetmf_op* op, const tetmf_mesh& m, bool device) {
  const int p = op->degree, nd = op->ndof;
  const int64_t nc = m.nc;
  auto nodes = library_nodes(p);
  // --- edges: sorted vertex pairs of all cells
  std::vector<uint64_t> ekeys;
  ekeys.reserve((size_t)6 * nc);
  const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  if (p >= 2)
    for (int64_t e = 0; e < nc; ++e)
      for (auto& ed : E) {
        uint64_t a = (uint32_t)m.tets[4 * e + ed[0]], b = (uint32_t)m.tets[4 * e + ed[1]];
        if (a > b) std::swap(a, b);
        ekeys.push_back(a << 32 | b);
      }
  std::sort(ekeys.begin(), ekeys.end());
  ekeys.erase(std::unique(ekeys.begin(), ekeys.end()), ekeys.end());
  const int64_t ne = (int64_t)ekeys.size();
  auto edge_id = [&](uint32_t a, uint32_t b) {
    if (a > b) std::swap(a, b);
    uint64_t k = (uint64_t)a << 32 | b;
    return (int64_t)(std::lower_bound(ekeys.begin(), ekeys.end(), k) - ekeys.begin());
  };
  // --- temporary DoF ids: vertices, edge nodes, face nodes
  const int64_t ntmp = m.nv + ne * (p - 1) + (p == 3 ? m.nf : 0);
  // boundary entities (Dirichlet constraints)
  std::vector<uint8_t> cons(ntmp, 0);
  if (op->bc == TETMF_DIRICHLET) {
    for (int64_t f = 0; f < m.nf; ++f) {
      if (m.fcell[2 * f + 1] >= 0) continue;
      const int32_t* t = &m.ftri[3 * f];
      for (int k = 0; k < 3; ++k) cons[t[k]] = 1;
      for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b) {
          int64_t eid = edge_id(t[a], t[b]);
          for (int k = 0; k < p - 1; ++k) cons[m.nv + eid * (p - 1) + k] = 1;
        }
      if (p == 3) cons[m.nv + ne * (p - 1) + f] = 1;
    }
  }
  const std::vector<int32_t>& perm = op->cell_perm;
  std::vector<int64_t> tmp((size_t)nc * nd);
  for (int64_t i = 0; i < nc; ++i) {
    const int64_t ue = perm[i];
    const int32_t* v = &m.tets[4 * ue];
    for (int j = 0; j < nd; ++j) {
      const auto& a = nodes[j];
      int nz = 0, idx[3];
      for (int k = 0; k < 4; ++k)
        if (a[k]) idx[nz++] = k;
      int64_t t;
      if (nz == 1) {
        t = v[idx[0]];
      } else if (nz == 2) {
        int va = v[idx[0]], vb = v[idx[1]];
        int mult_lo = va < vb ? a[idx[0]] : a[idx[1]];  // multiplicity at the smaller vertex id
        t = m.nv + edge_id(va, vb) * (p - 1) + (p - mult_lo - 1);
      } else {
        int opp = 0;
        for (int k = 0; k < 4; ++k)
          if (!a[k]) opp = k;
        t = m.nv + ne * (p - 1) + m.cell_face[4 * ue + opp];
      }
      tmp[(size_t)i * nd + j] = t;
    }
  }
  // --- blocks
  const int64_t nb = (nc + kBlockCells - 1) / kBlockCells;
  op->n_blocks = nb;
  op->ncp = nb * kBlockCells;
  // the kernels address the [n_dof][ncp] index arrays with 32-bit integers,
  // and read per-cell data with a 32-bit byte offset from a row base: at
  // most 4 rows of ncp values of 8 bytes (coefficients, geometry) or 16 rows
  // of 2-byte indices, i.e. below 32 ncp bytes
  const int64_t max_cells = std::min<int64_t>(INT32_MAX / nd, (int64_t)1 << 27) / kBlockCells * kBlockCells;
  if (op->ncp > max_cells)
    throw Error(TETMF_ERR_UNSUPPORTED, "mesh too large for one operator: at most " + std::to_string(max_cells) +
                                           " cells at this degree (32-bit indexing)");
  check_lane_maps((int)op->esize(), nd, op->nq, max_cells);
  std::vector<int32_t> bmin(ntmp, INT32_MAX), bmax(ntmp, -1);
  for (int64_t i = 0; i < nc; ++i) {
    int32_t b = (int32_t)(i / kBlockCells);
    for (int j = 0; j < nd; ++j) {
      int64_t t = tmp[(size_t)i * nd + j];
      bmin[t] = std::min(bmin[t], b);
      bmax[t] = std::max(bmax[t], b);
    }
  }
  // --- final numbering: per block, private DoFs (contiguous), then newly
  // touched shared free DoFs; constrained DoFs last.  Private DoFs are
  // ordered by the number of the block's cells that hold them (most first):
  // the kernels sum each DoF's slots in one lane, and a wave takes as many
  // steps as its longest sum, so DoFs with similar counts share a wave.
  std::vector<int64_t> gid(ntmp, -1);
  std::vector<int32_t> priv_start(nb), npriv(nb);
  std::vector<int32_t> mult(ntmp, 0);
  int64_t next = 0;
  for (int64_t b = 0; b < nb; ++b) {
    int64_t c0 = b * kBlockCells, c1 = std::min(nc, c0 + kBlockCells);
    priv_start[b] = (int32_t)next;
    std::vector<int64_t> cand;
    for (int64_t i = c0; i < c1; ++i)
      for (int j = 0; j < nd; ++j) {
        int64_t t = tmp[(size_t)i * nd + j];
        if (!cons[t] && bmin[t] == bmax[t] && mult[t]++ == 0) cand.push_back(t);
      }
    std::stable_sort(cand.begin(), cand.end(), [&](int64_t a, int64_t c) { return mult[a] > mult[c]; });
    for (int64_t t : cand) gid[t] = next++;
    npriv[b] = (int32_t)(next - priv_start[b]);
    for (int64_t i = c0; i < c1; ++i)
      for (int j = 0; j < nd; ++j) {
        int64_t t = tmp[(size_t)i * nd + j];
        if (gid[t] < 0 && !cons[t]) gid[t] = next++;
      }
  }
  op->n_free = next;
  for (int64_t i = 0; i < nc; ++i)
    for (int j = 0; j < nd; ++j) {
      int64_t t = tmp[(size_t)i * nd + j];
      if (gid[t] < 0) gid[t] = next++;
    }
  op->n_dofs = next;
  if (op->n_dofs > INT32_MAX) throw Error(TETMF_ERR_UNSUPPORTED, "more than 2^31 DoFs");
  // DoF values are staged with a 32-bit byte offset from the vector's start
  if ((uint64_t)op->n_dofs * op->esize() > UINT32_MAX)
    throw Error(TETMF_ERR_UNSUPPORTED, "too many DoFs for 32-bit byte offsets at this precision");
  // DoF coordinates and one containing cell
  op->dof_xyz.assign((size_t)3 * op->n_dofs, 0.0);
  op->dof_cell.assign(op->n_dofs, -1);
  for (int64_t i = 0; i < nc; ++i) {
    const int64_t ue = perm[i];
    for (int j = 0; j < nd; ++j) {
      int64_t g = gid[tmp[(size_t)i * nd + j]];
      if (op->dof_cell[g] >= 0) continue;
      op->dof_cell[g] = (int32_t)ue;
      for (int r = 0; r < 3; ++r) {
        double s = 0;
        for (int k = 0; k < 4; ++k) s += nodes[j][k] * m.xyz[3 * m.tets[4 * ue + k] + r];
        op->dof_xyz[3 * g + r] = s / p;
      }
    }
  }
  // shared free DoFs: ordered by global id, with the number of blocks touching each
  std::vector<int32_t> shared_index(op->n_dofs, -1);
  std::vector<int32_t> sh_gid;
  for (int64_t t = 0; t < ntmp; ++t)
    if (bmax[t] >= 0 && !cons[t] && bmin[t] != bmax[t]) sh_gid.push_back((int32_t)gid[t]);
  std::sort(sh_gid.begin(), sh_gid.end());
  for (size_t s = 0; s < sh_gid.size(); ++s) shared_index[sh_gid[s]] = (int32_t)s;
  op->n_shared = (int64_t)sh_gid.size();
  // --- per block lists
  std::vector<int32_t> blk_nbd(nb), blk_other_off(nb), blk_ptr_off(nb);
  std::vector<int32_t> other_gid, other_pslot;
  std::vector<uint16_t> slot_ptr;
  std::vector<uint16_t> lidx((size_t)nd * op->ncp, 0), pos((size_t)nd * op->ncp, 0);
  std::vector<int32_t> stamp(op->n_dofs, -1), local_of(op->n_dofs, 0), occ(op->n_dofs, 0);
  std::vector<int32_t> sh_count(sh_gid.size(), 0);
  std::vector<std::vector<int32_t>> block_shared(nb);
  int nbd_max = 0;
  for (int64_t b = 0; b < nb; ++b) {
    int64_t c0 = b * kBlockCells, c1 = std::min(nc, c0 + kBlockCells);
    int32_t nloc = npriv[b];
    std::vector<int32_t> others;
    for (int64_t i = c0; i < c1; ++i)
      for (int j = 0; j < nd; ++j) {
        int64_t g = gid[tmp[(size_t)i * nd + j]];
        if (stamp[g] == b) {
          if (local_of[g] < 0) occ[g]++;
          continue;
        }
        stamp[g] = (int32_t)b;
        if (g >= priv_start[b] && g < priv_start[b] + npriv[b]) {
          local_of[g] = (int32_t)(g - priv_start[b]);
        } else {
          local_of[g] = -1;
          occ[g] = 1;
          others.push_back((int32_t)g);
        }
      }
    // the block's other DoFs, likewise ordered by their number of slots here,
    // and by global id among equal counts: the partial sums of a block are
    // then written at increasing addresses within each count class
    std::sort(others.begin(), others.end(),
              [&](int32_t a, int32_t c) { return occ[a] > occ[c] || (occ[a] == occ[c] && a < c); });
    for (int32_t g : others) local_of[g] = nloc++;
    blk_nbd[b] = nloc;
    nbd_max = std::max(nbd_max, nloc);
    if (nloc > kBlockCells * nd) throw Error(TETMF_ERR_DEVICE, "internal: block DoF count overflow");
    // slots grouped by block DoF, cell-major inside a DoF
    std::vector<int32_t> cnt(nloc + 1, 0);
    for (int64_t i = c0; i < c1; ++i)
      for (int j = 0; j < nd; ++j) cnt[local_of[gid[tmp[(size_t)i * nd + j]]] + 1]++;
    for (int k = 0; k < nloc; ++k) cnt[k + 1] += cnt[k];
    blk_ptr_off[b] = (int32_t)slot_ptr.size();
    for (int k = 0; k <= nloc; ++k) slot_ptr.push_back((uint16_t)cnt[k]);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = c0; i < c1; ++i)
      for (int j = 0; j < nd; ++j) {
        int32_t l = local_of[gid[tmp[(size_t)i * nd + j]]];
        lidx[(size_t)j * op->ncp + i] = (uint16_t)l;
        pos[(size_t)j * op->ncp + i] = (uint16_t)fill[l]++;
      }
    blk_other_off[b] = (int32_t)other_gid.size();
    for (int32_t g : others) {
      other_gid.push_back(g);
      other_pslot.push_back(-1);
      if (g < op->n_free) {
        int32_t s = shared_index[g];
        sh_count[s]++;
        block_shared[b].push_back((int32_t)(other_gid.size() - 1));
      }
    }
  }
  // padding entry: every block's list offset stays a valid index
  other_gid.push_back(0);
  other_pslot.push_back(-1);
  std::vector<int32_t> sh_ptr(sh_gid.size() + 1, 0);
  for (size_t s = 0; s < sh_gid.size(); ++s) sh_ptr[s + 1] = sh_ptr[s] + sh_count[s];
  op->n_partials = sh_ptr.back();
  std::vector<int32_t> sh_fill(sh_ptr.begin(), sh_ptr.end() - 1);
  for (int64_t b = 0; b < nb; ++b)
    for (int32_t o : block_shared[b]) other_pslot[o] = sh_fill[shared_index[other_gid[o]]]++;
  std::string err = validate_cg(op, nd, priv_start, npriv, blk_nbd, blk_other_off, blk_ptr_off, other_gid,
                                other_pslot, lidx, pos, slot_ptr, sh_gid, sh_ptr, nbd_max);
  if (!err.empty()) throw Error(TETMF_ERR_DEVICE, "internal: " + err);
  if (!device) return;
  // --- device
  CGDev& d = op->cg;
  d.n_cell = (int)nc;
  d.ncp = (int)op->ncp;
  d.n_dofs = (int)op->n_dofs;
  d.n_free = (int)op->n_free;
  d.n_blocks = (int)nb;
  d.n_shared = (int)op->n_shared;
  d.nq = op->nq;
  d.nbd_max = nbd_max;
  d.sigma = op->sigma;
  d.curved = op->curved ? 1 : 0;
  d.ncomp = op->ncomp;
  d.geo = op->upload_real(op->curved ? point_geometry(op->qjac, perm, op->nq, op->ncp)
                                     : cell_geometry(m, perm, op->ncp));
  d.blk_priv_start = (const int*)op->upload(priv_start);
  d.blk_npriv = (const int*)op->upload(npriv);
  d.blk_nbd = (const int*)op->upload(blk_nbd);
  d.blk_other_off = (const int*)op->upload(blk_other_off);
  d.blk_ptr_off = (const int*)op->upload(blk_ptr_off);
  d.other_gid = (const int*)op->upload(other_gid);
  d.other_pslot = (const int*)op->upload(other_pslot);
  d.lidx = (const uint16_t*)op->upload(lidx);
  d.pos = (const uint16_t*)op->upload(pos);
  d.slot_ptr = (const uint16_t*)op->upload(slot_ptr);
  d.sh_gid = (const int*)op->upload(sh_gid);
  d.sh_ptr = (const int*)op->upload(sh_ptr);
  if (op->n_partials * op->ncomp > INT32_MAX) throw Error(TETMF_ERR_UNSUPPORTED, "too many partial sums");
  d.n_partials = (int)op->n_partials;
  d.partials = op->alloc((size_t)std::max<int64_t>(op->n_partials * op->ncomp, 1) * op->esize());
}

void setup_dg(tetmf_op* op, const tetmf_mesh& m, bool device) {
  const int p = op->degree, nd = op->ndof;
  const int64_t nc = m.nc;
  auto nodes = library_nodes(p);
  op->ncp = ((nc + kTile - 1) / kTile) * kTile;
  op->n_dofs = nc * nd;
  op->n_free = op->n_dofs;
  // DoF and per-cell array indices are 32-bit in the kernels
  if ((int64_t)nd * op->ncp > INT32_MAX) throw Error(TETMF_ERR_UNSUPPORTED, "more than 2^31 DoFs");
  const auto& perm = op->cell_perm;
  const auto& u2l = op->user_to_lib;
  op->dof_xyz.assign((size_t)3 * op->n_dofs, 0.0);
  op->dof_cell.assign(op->n_dofs, -1);
  for (int64_t i = 0; i < nc; ++i)
    for (int j = 0; j < nd; ++j) {
      op->dof_cell[i * nd + j] = perm[i];
      for (int r = 0; r < 3; ++r) {
        double s = 0;
        for (int k = 0; k < 4; ++k) s += nodes[j][k] * m.xyz[3 * m.tets[4 * (int64_t)perm[i] + k] + r];
        op->dof_xyz[3 * (i * nd + j) + r] = s / p;
      }
    }
  // node permutation of every relabelling: relabelled node k (multi-index b
  // over the relabelled vertices) is the original node with a[s[i]] = b[i].
  auto rel = all_relabellings();
  std::vector<uint8_t> ptab((size_t)24 * nd);
  for (int r = 0; r < 24; ++r)
    for (int k = 0; k < nd; ++k) {
      std::array<int, 4> a{};
      for (int i = 0; i < 4; ++i) a[rel[r][i]] = nodes[k][i];
      int found = -1;
      for (int j = 0; j < nd; ++j)
        if (nodes[j] == a) found = j;
      ptab[(size_t)r * nd + k] = (uint8_t)found;
    }
  // face data per (local face f, library cell i)
  const int64_t ncp = op->ncp;
  std::vector<int32_t> nb((size_t)4 * ncp, -1), fid((size_t)4 * ncp, 0), code((size_t)4 * ncp, 0);
  std::vector<double> fgeo((size_t)8 * 4 * ncp, 0.0);
  const double pen = op->eta * (p + 1) * (p + 1);
  auto relabel_for = [&](int64_t ue, int f, const int32_t* tri) {
    // relabelled vertices (a, b, c, opposite) as local indices of cell ue
    std::array<int, 4> s{};
    const int32_t* v = &m.tets[4 * ue];
    for (int k = 0; k < 3; ++k)
      for (int i = 0; i < 4; ++i)
        if (v[i] == tri[k]) s[k] = i;
    s[3] = f;
    return s;
  };
  for (int64_t i = 0; i < nc; ++i) {
    const int64_t ue = perm[i];
    for (int f = 0; f < 4; ++f) {
      const int32_t F = m.cell_face[4 * ue + f];
      const int32_t* tri = &m.ftri[3 * (int64_t)F];
      int32_t c0 = m.fcell[2 * F], c1 = m.fcell[2 * F + 1];
      int64_t other = (c0 == ue) ? c1 : c0;
      int other_local = (c0 == ue) ? m.flocal[2 * F + 1] : m.flocal[2 * F];
      auto so = relabel_for(ue, f, tri);
      // geometry of the face
      const double* A = &m.xyz[3 * tri[0]];
      const double* B = &m.xyz[3 * tri[1]];
      const double* C = &m.xyz[3 * tri[2]];
      double ab[3], ac[3], nrm[3];
      for (int r = 0; r < 3; ++r) {
        ab[r] = B[r] - A[r];
        ac[r] = C[r] - A[r];
      }
      nrm[0] = ab[1] * ac[2] - ab[2] * ac[1];
      nrm[1] = ab[2] * ac[0] - ab[0] * ac[2];
      nrm[2] = ab[0] * ac[1] - ab[1] * ac[0];
      double len = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
      double area = 0.5 * len;
      for (int r = 0; r < 3; ++r) nrm[r] /= len;
      const double* O = &m.xyz[3 * m.tets[4 * ue + f]];
      double side = 0;
      for (int r = 0; r < 3; ++r) side += (O[r] - A[r]) * nrm[r];
      if (side > 0)
        for (int r = 0; r < 3; ++r) nrm[r] = -nrm[r];  // outward from the own cell
      auto bvec = [&](const double* opp, double out[3]) {
        M3 Js;
        for (int r = 0; r < 3; ++r) {
          Js.a[r][0] = ab[r];
          Js.a[r][1] = ac[r];
          Js.a[r][2] = opp[r] - A[r];
        }
        M3 Ji = inv3(Js);
        for (int r = 0; r < 3; ++r) out[r] = Ji.a[r][0] * nrm[0] + Ji.a[r][1] * nrm[1] + Ji.a[r][2] * nrm[2];
      };
      double bo[3], bn[3] = {0, 0, 0};
      bvec(O, bo);
      int code_nb = 0;
      double tau;
      if (other >= 0) {
        auto sn = relabel_for(other, other_local, tri);
        code_nb = relabelling_id(sn);
        bvec(&m.xyz[3 * m.tets[4 * other + other_local]], bn);
        nb[(size_t)f * ncp + i] = u2l[other];
        tau = pen * area / std::min(m.vol[ue], m.vol[other]);
      } else {
        tau = pen * area / m.vol[ue];
      }
      fid[(size_t)f * ncp + i] = F;
      code[(size_t)f * ncp + i] = relabelling_id(so) | (code_nb << 8);
      const double vals[8] = {bo[0], bo[1], bo[2], bn[0], bn[1], bn[2], 2.0 * area, tau};
      for (int k = 0; k < 8; ++k) fgeo[((size_t)k * 4 + f) * ncp + i] = vals[k];
    }
  }
  // host invariants the DG kernel relies on for its memory accesses
  for (size_t i = 0; i < ptab.size(); ++i)
    if (ptab[i] >= nd) throw Error(TETMF_ERR_DEVICE, "internal: node permutation table");
  for (int64_t f = 0; f < 4; ++f)
    for (int64_t i = 0; i < nc; ++i) {
      const size_t x = (size_t)f * ncp + i;
      if (nb[x] >= nc || fid[x] < 0 || fid[x] >= m.nf || (code[x] & 255) >= 24 || (code[x] >> 8) >= 24)
        throw Error(TETMF_ERR_DEVICE, "internal: face data of cell " + std::to_string(i));
    }
  if (!device) return;
  DGDev& d = op->dg;
  d.n_cell = (int)nc;
  d.ncp = (int)ncp;
  d.n_face = (int)m.nf;
  d.nq = op->nq;
  d.nqf = op->nqf;
  d.dirichlet = op->bc == TETMF_DIRICHLET;
  d.sigma = op->sigma;
  d.geo = op->upload_real(cell_geometry(m, perm, ncp));
  d.nb = (const int*)op->upload(nb);
  d.fid = (const int*)op->upload(fid);
  d.code = (const int*)op->upload(code);
  d.fgeo = op->upload_real(fgeo);
  d.perm = (const uint8_t*)op->upload(ptab);
}

// Algorithmic work of one apply with a per-point coefficient: the paper's
// counts eq. (8)-(11) adapted to a coefficient per quadrature point and a
// mass term (r = 4 tabulated rows per point instead of 3), vectors read once
// and written once (no read-for-ownership).
void work_model(tetmf_op* op, const tetmf_mesh& m) {
  const double s = op->prec == TETMF_F64 ? 8.0 : 4.0;
  const double nq = op->nq, nd = op->ndof;
  const bool mass = op->sigma != 0.0;
  const double r = mass ? 4 : 3;
  const double cq = mass ? 37 : 34;
  const double fcell = 4 * r * nq * nd + cq * nq + nd;
  if (op->kind == TETMF_CG) {
    // geometry per cell, or per rule point for curved cells; a vector field
    // reads the cell data once and its components' vectors each once
    const double ng = (mass ? 7 : 6) * (op->curved ? nq : 1.0);
    op->flops = fcell * m.nc * op->ncomp;
    op->bytes = m.nc * (ng * s + 4 * nd + s * nq) + 2 * s * (double)op->nvec();
    // backward: u and g interpolated, D applied to g and integrated (du),
    // plus w_q grad u . G grad g per point (21 flops); kappa read, dkappa
    // written, u and g read, du written
    op->flops_bwd = (6 * r * nq * nd + (cq + 21) * nq + nd) * m.nc * op->ncomp;
    op->bytes_bwd = m.nc * (ng * s + 4 * nd + 2 * s * nq) + 3 * s * (double)op->nvec();
  } else {
    const double nqf = op->nqf;
    const double nbf = (double)(m.nf - m.nif);
    // a vector field runs one full pass per component
    op->flops = op->ncomp * (fcell * m.nc + m.nif * (32 * nqf * nd + 46 * nqf) +
                             (op->bc == TETMF_DIRICHLET ? nbf * (16 * nqf * nd + 30 * nqf) : 0.0));
    op->bytes = op->ncomp * (m.nc * (7 * s + s * nq + 20 + 2 * s * nd) + m.nf * (s * nqf + 8));
    // backward: du = A g (one apply) and the coefficient-gradient pass, which
    // interpolates u and g at the cell points (21 flops each for dkappa) and
    // both traces of u and g at the face points (4 values of nd terms per
    // side and field), with about 30 (interior) / 20 (boundary) flops of the
    // flux bracket per face point; it reads both coefficients and writes
    // their gradients
    const double fgrad = m.nc * (4 * r * nq * nd + 21 * nq) + m.nif * (32 * nqf * nd + 30 * nqf) +
                         (op->bc == TETMF_DIRICHLET ? nbf * (16 * nqf * nd + 20 * nqf) : 0.0);
    const double bgrad = m.nc * (7 * s + 2 * s * nq + 20 + 2 * s * nd) + m.nf * (2 * s * nqf + 8);
    op->flops_bwd = op->flops + op->ncomp * fgrad;
    op->bytes_bwd = op->bytes + op->ncomp * bgrad;
  }
}

}  // namespace

namespace {

// Argument checks and the host-side fields of an op (no device access).
int init_op(const tetmf_mesh* mesh, const tetmf_op_desc* d, tetmf_op* op, const char* who) {
  const std::string w(who);
  if (d->kind != TETMF_CG && d->kind != TETMF_DG) return fail(TETMF_ERR_INVALID_ARGUMENT, w + ": kind must be CG or DG");
  if (d->degree < 1 || d->degree > 3) return fail(TETMF_ERR_UNSUPPORTED, w + ": degree must be 1..3");
  if (d->precision < TETMF_F64 || d->precision > TETMF_BF16IN) return fail(TETMF_ERR_INVALID_ARGUMENT, w + ": bad precision");
  if (d->bc != TETMF_NEUMANN && d->bc != TETMF_DIRICHLET)
    return fail(TETMF_ERR_INVALID_ARGUMENT, w + ": bad boundary condition");
  if (d->ordering != TETMF_ORDER_LOCALITY && d->ordering != TETMF_ORDER_AS_GIVEN)
    return fail(TETMF_ERR_INVALID_ARGUMENT, w + ": bad ordering");
  if (d->n_q < 1 || !d->q_points || !d->q_weights)
    return fail(TETMF_ERR_INVALID_ARGUMENT, w + ": missing cell quadrature rule");
  if (d->kind == TETMF_DG && (d->n_qf < 1 || !d->qf_points || !d->qf_weights))
    return fail(TETMF_ERR_INVALID_ARGUMENT, w + ": missing face quadrature rule");
  if (!std::isfinite(d->sigma) || d->sigma < 0 || !std::isfinite(d->eta) || d->eta <= 0)
    return fail(TETMF_ERR_INVALID_ARGUMENT, w + ": sigma must be >= 0 and eta > 0");
  op->kind = d->kind;
  op->degree = d->degree;
  op->bc = d->bc;
  op->prec = d->precision;
  op->device = d->device;
  op->ndof = (d->degree + 1) * (d->degree + 2) * (d->degree + 3) / 6;
  op->nq = d->n_q;
  op->nqf = d->kind == TETMF_DG ? d->n_qf : 0;
  op->mt = mt_for(op->nq);
  op->mtf = op->nqf ? mt_for(op->nqf) : 0;
  op->sigma = d->sigma;
  op->eta = d->eta;
  op->nc = mesh->nc;
  op->nf = mesh->nf;
  op->nif = mesh->nif;
  op->mesh_tag = mesh;
  op->mesh_nc = mesh->nc;
  op->mesh_nv = mesh->nv;
  // compiled kernel shapes: (DoFs per cell, cell points[, face points])
  bool ok;
  if (op->kind == TETMF_CG)
    ok = (op->ndof == 4 && op->nq == 4) || (op->ndof == 10 && (op->nq == 4 || op->nq == 14)) ||
         (op->ndof == 20 && (op->nq == 14 || op->nq == 24));
  else
    ok = (op->ndof == 4 && op->nq == 4 && op->nqf == 3) || (op->ndof == 10 && op->nq == 14 && op->nqf == 6) ||
         (op->ndof == 20 && op->nq == 24 && op->nqf == 12);
  if (op->kind == TETMF_DG && op->prec == TETMF_BF16IN) ok = false;
  if (!ok)
    return fail(TETMF_ERR_UNSUPPORTED, w + ": no kernel for degree " + std::to_string(op->degree) + " with " +
                                           std::to_string(op->nq) + " cell / " + std::to_string(op->nqf) +
                                           " face points");
  for (int q = 0; q < op->nq; ++q) {
    const double* x = &d->q_points[3 * q];
    if (!(x[0] >= 0 && x[1] >= 0 && x[2] >= 0 && x[0] + x[1] + x[2] <= 1) || !(d->q_weights[q] > 0))
      return fail(TETMF_ERR_INVALID_ARGUMENT, w + ": quadrature point outside the reference cell");
  }
  if (d->n_components != 0 && d->n_components != 1 && d->n_components != 3)
    return fail(TETMF_ERR_UNSUPPORTED, w + ": n_components must be 1 or 3");
  if (d->n_components == 3) {
    if (op->prec == TETMF_BF16IN)
      return fail(TETMF_ERR_UNSUPPORTED, w + ": vector fields are supported in FP64 and FP32 only");
    op->ncomp = 3;
  }
  if (d->q_jacobians) {
    if (op->kind != TETMF_CG) return fail(TETMF_ERR_UNSUPPORTED, w + ": curved cells are supported for CG only");
    for (int64_t e = 0; e < mesh->nc; ++e)
      for (int q = 0; q < op->nq; ++q) {
        const double* a = &d->q_jacobians[((size_t)e * op->nq + q) * 9];
        M3 J;
        double fro = 0;
        bool finite = true;
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) {
            J.a[r][c] = a[3 * r + c];
            fro += a[3 * r + c] * a[3 * r + c];
            finite = finite && std::isfinite(a[3 * r + c]);
          }
        const double det = finite ? std::fabs(det3(J)) : 0.0;
        if (!finite || !(det > 1e-12 * fro * std::sqrt(fro)))
          return fail(TETMF_ERR_DEGENERATE_CELL, w + ": degenerate or non-finite Jacobian at cell " +
                                                     std::to_string(e) + ", point " + std::to_string(q));
      }
    op->curved = true;
    op->qjac = d->q_jacobians;
  }
  if (d->ordering == TETMF_ORDER_AS_GIVEN) {
    op->cell_perm.resize(mesh->nc);
    std::iota(op->cell_perm.begin(), op->cell_perm.end(), 0);
  } else {
    op->cell_perm = locality_order(*mesh);
  }
  op->user_to_lib.assign(mesh->nc, 0);
  for (int64_t i = 0; i < mesh->nc; ++i) op->user_to_lib[op->cell_perm[i]] = (int32_t)i;
  return TETMF_OK;
}

}  // namespace

extern "C" int tetmf_op_create(const tetmf_mesh* mesh, const tetmf_op_desc* d, tetmf_op** out) {
  return guarded([&]() -> int {
    if (!mesh || !d || !out) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_op_create: NULL argument");
    *out = nullptr;
    int ndev = 0;
    check_hip(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (d->device < 0 || d->device >= ndev) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_op_create: bad device");
    int prev = 0;
    check_hip(hipGetDevice(&prev), "hipGetDevice");
    check_hip(hipSetDevice(d->device), "hipSetDevice");
    struct Restore {
      int dev;
      ~Restore() { (void)hipSetDevice(dev); }
    } restore{prev};
    auto op = new tetmf_op();
    std::unique_ptr<tetmf_op> guard(op);
    int st = init_op(mesh, d, op, "tetmf_op_create");
    if (st) return st;
    op->d_cell_perm = (int32_t*)op->upload(op->cell_perm);
    if (op->kind == TETMF_CG) {
      setup_cg(op, *mesh, true);
      // device address of the fixed scratch of tetmf_apply_noalloc on this
      // device (resolved once per device, with the device current)
      void* scr = nullptr;
      check_hip(noalloc_scratch(&scr), "scratch symbol address");
    } else {
      setup_dg(op, *mesh, true);
    }
    fill_tables(op, d);
    work_model(op, *mesh);
    op->qjac = nullptr;
    *out = guard.release();
    return TETMF_OK;
  });
}

extern "C" int tetmf_op_check(const tetmf_mesh* mesh, const tetmf_op_desc* d, int64_t* n_dofs, int64_t* n_free) {
  return guarded([&]() -> int {
    if (!mesh || !d) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_op_check: NULL argument");
    tetmf_op op;
    int st = init_op(mesh, d, &op, "tetmf_op_check");
    if (st) return st;
    if (op.kind == TETMF_CG)
      setup_cg(&op, *mesh, false);
    else
      setup_dg(&op, *mesh, false);
    if (n_dofs) *n_dofs = op.n_dofs;
    if (n_free) *n_free = op.n_free;
    return TETMF_OK;
  });
}

extern "C" void tetmf_op_destroy(tetmf_op* op) { delete op; }

extern "C" int tetmf_op_info(const tetmf_op* op, tetmf_info* info) {
  if (!op || !info) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_op_info: NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->n_dofs = op->n_dofs;
  info->n_components = op->ncomp;
  info->n_free = op->n_free;
  info->n_cell = op->nc;
  info->n_face = op->nf;
  info->n_interior_face = op->nif;
  info->n_q = op->nq;
  info->n_qf = op->nqf;
  info->n_dof_cell = op->ndof;
  info->precision = op->prec;
  info->n_blocks = op->n_blocks;
  info->n_shared = op->n_shared;
  info->n_partials = op->n_partials;
  info->flops_per_apply = op->flops;
  info->bytes_per_apply = op->bytes;
  info->device_bytes = op->device_bytes();
  info->flops_per_backward = op->flops_bwd;
  info->bytes_per_backward = op->bytes_bwd;
  info->n_cell_data = lanes::cell_data_size(op->nq, op->nc);
  return TETMF_OK;
}

extern "C" int tetmf_op_numbering(const tetmf_op* op, int32_t* cell_perm, double* dof_xyz, int32_t* dof_cell) {
  if (!op) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_op_numbering: NULL op");
  if (cell_perm) std::memcpy(cell_perm, op->cell_perm.data(), op->cell_perm.size() * sizeof(int32_t));
  if (dof_xyz) std::memcpy(dof_xyz, op->dof_xyz.data(), op->dof_xyz.size() * sizeof(double));
  if (dof_cell) std::memcpy(dof_cell, op->dof_cell.data(), op->dof_cell.size() * sizeof(int32_t));
  return TETMF_OK;
}

namespace {

struct DeviceScope {
  int prev = 0;
  explicit DeviceScope(int dev) {
    check_hip(hipGetDevice(&prev), "hipGetDevice");
    if (prev != dev) check_hip(hipSetDevice(dev), "hipSetDevice");
  }
  ~DeviceScope() { (void)hipSetDevice(prev); }
};

int kernel_prec(const tetmf_op* op) {
  return op->prec == TETMF_F64 ? PREC_F64 : op->prec == TETMF_F32 ? PREC_F32 : PREC_BF16;
}

int run_cg(tetmf_op* op, int mode, const void* u, const void* g, const void* kappa, void* out, void* dk,
           void* stream) {
  DeviceScope ds(op->device);
  bool supported = true;
  hipError_t e = launch_cg(op->cg, kernel_prec(op), op->ndof, op->nq, mode, u, g, kappa, out, dk,
                           (hipStream_t)stream, &supported, op->next_events());
  if (!supported) return fail(TETMF_ERR_UNSUPPORTED, "no kernel instantiation for this operator");
  check_hip(e, "kernel launch");
  return TETMF_OK;
}

// Operator diagonal; every component of a vector field has the scalar
// operator's diagonal.
int run_diag(tetmf_op* op, const void* kappa, void* d, void* stream) {
  int st = run_cg(op, MODE_DIAG, nullptr, nullptr, kappa, d, nullptr, stream);
  for (int c = 1; c < op->ncomp && st == TETMF_OK; ++c)
    check_hip(hipMemcpyAsync((char*)d + (size_t)c * op->n_dofs * op->esize(), d, (size_t)op->n_dofs * op->esize(),
                             hipMemcpyDeviceToDevice, (hipStream_t)stream),
              "hipMemcpyAsync");
  return st;
}

}  // namespace

extern "C" int tetmf_cell_data_layout(const tetmf_op* op, const void* src, void* dst, int to_user, void* stream) {
  return guarded([&]() -> int {
    if (!op || !src || !dst) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_cell_data_layout: NULL argument");
    if (src == dst) return fail(TETMF_ERR_ALIAS, "tetmf_cell_data_layout: src and dst alias");
    DeviceScope ds(op->device);
    check_hip(launch_layout(kernel_prec(op), to_user, op->d_cell_perm, (int)op->nc, op->nq, src, dst,
                            (hipStream_t)stream),
              "layout kernel");
    return TETMF_OK;
  });
}

extern "C" int tetmf_apply(tetmf_op* op, const void* u, const void* kappa_cell, const void* kappa_face, void* v,
                           void* stream) {
  return guarded([&]() -> int {
    if (!op || !u || !v) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_apply: NULL op or vector");
    if (u == v) return fail(TETMF_ERR_ALIAS, "tetmf_apply: u and v alias");
    if (op->kind == TETMF_CG) {
      if (kappa_face) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_apply: kappa_face given for a CG operator");
      return run_cg(op, MODE_APPLY, u, nullptr, kappa_cell, v, nullptr, stream);
    }
    DeviceScope ds(op->device);
    bool supported = true;
    // SIPG is cell-local: a vector field is one pass per component
    const size_t cstride = (size_t)op->n_dofs * op->esize();
    for (int c = 0; c < op->ncomp; ++c) {
      hipError_t e = launch_dg(op->dg, kernel_prec(op), op->ndof, op->nq, op->nqf, (const char*)u + c * cstride,
                               kappa_cell, kappa_face, (char*)v + c * cstride, (hipStream_t)stream, &supported,
                               op->next_events());
      if (!supported) return fail(TETMF_ERR_UNSUPPORTED, "no DG kernel instantiation for this operator");
      check_hip(e, "kernel launch");
    }
    return TETMF_OK;
  });
}

extern "C" int tetmf_apply_noalloc(tetmf_op* op, const void* u, const void* kappa_cell, const void* kappa_face,
                                   void* v, void* stream) {
  return guarded([&]() -> int {
    if (!op || !u || !v) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_apply_noalloc: NULL op or vector");
    if (u == v) return fail(TETMF_ERR_ALIAS, "tetmf_apply_noalloc: u and v alias");
    DeviceScope ds(op->device);
    bool supported = true;
    if (op->kind != TETMF_CG) {
      // SIPG is cell-local and uses no scratch: the launches of tetmf_apply
      const size_t cstride = (size_t)op->n_dofs * op->esize();
      for (int c = 0; c < op->ncomp; ++c) {
        hipError_t e = launch_dg(op->dg, kernel_prec(op), op->ndof, op->nq, op->nqf, (const char*)u + c * cstride,
                                 kappa_cell, kappa_face, (char*)v + c * cstride, (hipStream_t)stream, &supported,
                                 nullptr);
        if (!supported) return fail(TETMF_ERR_UNSUPPORTED, "no DG kernel instantiation for this operator");
        check_hip(e, "kernel launch");
      }
      return TETMF_OK;
    }
    if (kappa_face) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_apply_noalloc: kappa_face given for a CG operator");
    const uint64_t need = (uint64_t)op->n_partials * (uint64_t)op->ncomp * (uint64_t)op->esize();
    if (need > (uint64_t)TETMF_NOALLOC_SCRATCH_BYTES)
      return fail(TETMF_ERR_UNSUPPORTED, "tetmf_apply_noalloc: the operator needs " + std::to_string(need) +
                                             " bytes of interface partial sums, more than the fixed scratch of " +
                                             std::to_string((uint64_t)TETMF_NOALLOC_SCRATCH_BYTES) +
                                             " bytes; use tetmf_apply");
    void* scr = nullptr;
    check_hip(noalloc_scratch(&scr), "scratch symbol address");
    // the op's kernels with the partial sums in the fixed scratch
    CGDev d = op->cg;
    d.partials = scr;
    hipError_t e = launch_cg(d, kernel_prec(op), op->ndof, op->nq, MODE_APPLY, u, nullptr, kappa_cell, v, nullptr,
                             (hipStream_t)stream, &supported, nullptr);
    if (!supported) return fail(TETMF_ERR_UNSUPPORTED, "no kernel instantiation for this operator");
    check_hip(e, "kernel launch");
    return TETMF_OK;
  });
}

extern "C" int tetmf_apply_backward(tetmf_op* op, const void* u, const void* g, const void* kappa_cell,
                                    const void* kappa_face, void* du, void* dkappa_cell, void* dkappa_face,
                                    void* stream) {
  return guarded([&]() -> int {
    if (!op || !u || !g) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_apply_backward: NULL argument");
    if (op->kind == TETMF_CG && (kappa_face || dkappa_face))
      return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_apply_backward: face coefficients given for a CG operator");
    if (du && (du == u || du == g)) return fail(TETMF_ERR_ALIAS, "tetmf_apply_backward: du aliases an input");
    if ((dkappa_cell && (dkappa_cell == u || dkappa_cell == g || dkappa_cell == du)) ||
        (dkappa_face && (dkappa_face == u || dkappa_face == g || dkappa_face == du || dkappa_face == dkappa_cell)))
      return fail(TETMF_ERR_ALIAS, "tetmf_apply_backward: an output aliases another argument");
    if (op->prec == TETMF_BF16IN) return fail(TETMF_ERR_UNSUPPORTED, "tetmf_apply_backward: BF16 operands");
    if (dkappa_cell && op->nc % 16 != 0) {
      // the padding cells of the last 16-cell tile get zeros (the kernels
      // write real cells only); a fill kernel, so that the call stays
      // capturable in a HIP graph
      DeviceScope dsz(op->device);
      const long last = lanes::cell_data_index(op->nq, 0, op->nc & ~(int64_t)15);
      check_hip(vec_fill(kernel_prec(op), (char*)dkappa_cell + last * op->esize(), 0.0, 16L * op->nq,
                         (hipStream_t)stream),
                "fill");
    }
    if (op->kind == TETMF_CG) {
      if (!du && !dkappa_cell) return TETMF_OK;
      return run_cg(op, MODE_BACKWARD, u, g, kappa_cell, du, dkappa_cell, stream);
    }
    // SIPG: A is symmetric, so du = A g is one forward apply; the coefficient
    // gradients come from one pass over cells and faces.
    DeviceScope ds(op->device);
    hipStream_t s = (hipStream_t)stream;
    bool supported = true;
    // vector fields: one pass per component; the coefficient gradients of
    // the later components are added to the first one's (component order)
    const size_t cstride = (size_t)op->n_dofs * op->esize();
    for (int c = 0; c < op->ncomp; ++c) {
      const char* uc = (const char*)u + c * cstride;
      const char* gc = (const char*)g + c * cstride;
      if (du) {
        hipError_t e = launch_dg(op->dg, kernel_prec(op), op->ndof, op->nq, op->nqf, gc, kappa_cell, kappa_face,
                                 (char*)du + c * cstride, s, &supported, nullptr);
        if (!supported) return fail(TETMF_ERR_UNSUPPORTED, "no DG kernel instantiation for this operator");
        check_hip(e, "kernel launch");
      }
      if (dkappa_cell || dkappa_face) {
        hipError_t e = launch_dg_grad(op->dg, kernel_prec(op), op->ndof, op->nq, op->nqf, uc, gc, dkappa_cell,
                                      dkappa_face, c > 0, s, &supported);
        if (!supported) return fail(TETMF_ERR_UNSUPPORTED, "no DG kernel instantiation for this operator");
        check_hip(e, "kernel launch");
      }
    }
    return TETMF_OK;
  });
}

extern "C" int tetmf_diagonal(tetmf_op* op, const void* kappa_cell, const void* kappa_face, void* d, void* stream) {
  return guarded([&]() -> int {
    if (!op || !d) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_diagonal: NULL argument");
    if (op->kind != TETMF_CG || kappa_face) return fail(TETMF_ERR_UNSUPPORTED, "tetmf_diagonal: only CG operators");
    return run_diag(op, kappa_cell, d, stream);
  });
}

extern "C" int tetmf_load_vector(tetmf_op* op, const void* f, void* b, void* stream) {
  return guarded([&]() -> int {
    if (!op || !b) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_load_vector: NULL argument");
    if (op->kind != TETMF_CG) return fail(TETMF_ERR_UNSUPPORTED, "tetmf_load_vector: only CG operators");
    if (op->ncomp != 1) return fail(TETMF_ERR_UNSUPPORTED, "tetmf_load_vector: scalar fields only");
    return run_cg(op, MODE_LOAD, nullptr, nullptr, f, b, nullptr, stream);
  });
}

// ---------------------------------------------------------------------------
// solver

namespace {

struct SolveScratch {
  void* v[8];
  double* scal;  // device scalars
  double* part;  // dot partials
};

double read_scalar(const double* d, hipStream_t s) {
  double h = 0;
  check_hip(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  return h;
}

// Preconditioned conjugate gradients on op: solves A d = rhs from d = 0 with
// fused vector kernels and device-resident scalars; the host reads r.r (one
// synchronisation) every kCheckEvery iterations, so up to kCheckEvery - 1
// iterations may run past the target.  Vectors are in the op precision; dot
// products accumulate in FP64.  Returns the iterations run.
constexpr int kCheckEvery = 4;

int pcg(tetmf_op* op, const void* kappa, const void* rhs, void* xsol, void* r, void* z, void* pv, void* q,
        const void* dinv, double* scal, double* part, double rtol_abs2, int max_it, hipStream_t s) {
  const int kp = kernel_prec(op);
  const int64_t n = op->nvec();
  double* rz = scal + 0;  // rz[0], rz[1]: double buffer
  double* rr = scal + 2;
  check_hip(pcg_init(kp, rhs, dinv, xsol, r, z, pv, part, rz, rr, n, s), "pcg init");
  if (read_scalar(rr, s) <= rtol_abs2) return 0;
  int it = 0;
  while (it < max_it) {
    int st = run_cg(op, MODE_APPLY, pv, nullptr, kappa, q, nullptr, s);
    if (st) throw Error(st, g_last_error);
    check_hip(pcg_iteration(kp, xsol, r, z, pv, q, dinv, part, rz + (it & 1), rz + ((it + 1) & 1), rr, nullptr, n, s),
              "pcg iteration");
    ++it;
    if ((it % kCheckEvery == 0 || it == max_it) && read_scalar(rr, s) <= rtol_abs2) break;
  }
  return it;
}

}  // namespace

extern "C" int tetmf_solve(tetmf_op* op64, const void* kappa64, tetmf_op* opi, const void* kappai, const double* b,
                           double* x, const tetmf_solve_opts* opts, tetmf_solve_stats* stats, void* stream) {
  return guarded([&]() -> int {
    if (!op64 || !b || !x || !opts) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_solve: NULL argument");
    if (op64->kind != TETMF_CG || op64->prec != TETMF_F64)
      return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_solve: op64 must be a CG FP64 operator");
    if (opi && (opi->kind != TETMF_CG || opi->n_dofs != op64->n_dofs || opi->mesh_nc != op64->mesh_nc ||
                opi->cell_perm != op64->cell_perm || opi->n_free != op64->n_free || opi->curved != op64->curved ||
                opi->ncomp != op64->ncomp))
      return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_solve: inner operator does not match op64");
    if ((const void*)b == (const void*)x) return fail(TETMF_ERR_ALIAS, "tetmf_solve: b and x alias");
    if (opts->method != 0 && opts->method != 1)
      return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_solve: method must be 0 or 1");
    DeviceScope dsc(op64->device);
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    const int64_t n = op64->nvec();
    // scratch: FP64 residual + FP64 correction workspace + inner vectors
    tetmf_op* ow = opi ? opi : op64;
    if (op64->solve_bufs.empty()) {
      auto al = [&](size_t bytes) {
        void* p = nullptr;
        check_hip(hipMalloc(&p, std::max<size_t>(bytes, 16)), "hipMalloc");
        op64->solve_bufs.push_back({p, bytes});
        return p;
      };
      for (int i = 0; i < 2; ++i) al(n * 8);          // r64, tmp64
      for (int i = 0; i < 6; ++i) al(n * 8);          // inner vectors (sized for FP64)
      al(64 * sizeof(double));                        // scalars
      al(4096 * sizeof(double));                      // dot partials
    }
    auto& sb = op64->solve_bufs;
    double* r64 = (double*)sb[0].p;
    double* tmp64 = (double*)sb[1].p;
    void* ir = sb[2].p;
    void* iz = sb[3].p;
    void* ip = sb[4].p;
    void* iq = sb[5].p;
    void* id = sb[6].p;   // inner solution d
    void* idinv = sb[7].p;
    double* scal = (double*)sb[8].p;
    double* part = (double*)sb[9].p;
    const int kpi = kernel_prec(ow);
    // Jacobi preconditioner of the inner operator
    if (opts->precond == 1) {
      int st = run_diag(ow, opi ? kappai : kappa64, idinv, s);
      if (st) return st;
      check_hip(vec_recip(kpi, idinv, n, s), "recip");
    } else {
      check_hip(vec_fill(kpi, idinv, 1.0, n, s), "fill");
    }
    check_hip(vec_dot(PREC_F64, b, b, n, part, scal + 10, s), "dot");
    const double bnorm2 = read_scalar(scal + 10, s);
    const double tol2 = opts->rtol * opts->rtol * bnorm2;
    // Method 0 and the plain FP64 PCG: the FP64 true residual r = b - A64 x,
    // then a Jacobi-PCG solve of A_inner d = r and x += d.  With an inner
    // operator the inner solve stops at inner_rtol ||r|| (iterative
    // refinement); without one it runs in FP64 down to rtol ||b|| / 2, so that
    // its recursion-vs-true residual gap stays below the target, and the outer
    // loop only confirms (or repeats).  Method 1: below.
    int outer = 0, inner_total = 0, status = TETMF_NOT_CONVERGED;
    double relres = 1.0;
    const int max_outer = std::max(1, opts->max_outer);
    // FP64 true residual r64 = b - A64 x, its squared norm, relres
    auto true_residual = [&]() -> double {
      int st = run_cg(op64, MODE_APPLY, x, nullptr, kappa64, tmp64, nullptr, s);
      if (st) throw Error(st, g_last_error);
      check_hip(vec_sub(b, tmp64, r64, n, s), "sub");
      check_hip(vec_dot(PREC_F64, r64, r64, n, part, scal + 11, s), "dot");
      const double rn2 = read_scalar(scal + 11, s);
      relres = bnorm2 > 0 ? std::sqrt(rn2 / bnorm2) : std::sqrt(rn2);
      return rn2;
    };
    if (opi && opts->method == 1) {
      // Reliable updates: one inner-precision PCG on A_inner d = r (d in id,
      // added to x in FP64 at every replacement).  Its residual is replaced by
      // the cast FP64 true residual when the recursive one has fallen by
      // inner_rtol since the last replacement, or below rtol ||b|| / 2; the
      // search direction p is kept, and the new r.z enters the next step's
      // alpha and beta.  The direction is kept only for an FP32 inner
      // operator and while the true residual agrees with the recursive one
      // (squared norms within a factor 4); BF16 operands (products symmetric
      // only to their rounding, about 3e-3) restart it at every replacement,
      // which makes each step an iterative-refinement step (a kept direction
      // stalled their recursion).  A non-finite recursive residual discards
      // the inner iterate and restarts from x.
      double rn2 = true_residual();
      const double red2 = opts->inner_rtol * opts->inner_rtol;
      const int max_inner = std::max(1, opts->max_inner);
      double* rz = scal + 0;  // double-buffered r.z (iteration it reads rz[it & 1])
      double* rr = scal + 2;
      int it = 0;
      if (rn2 <= tol2) {
        status = TETMF_OK;
      } else {
        check_hip(vec_cast(PREC_F64, r64, kpi, iq, n, s), "cast");
        check_hip(pcg_init(kpi, iq, idinv, id, ir, iz, ip, part, rz, rr, n, s), "pcg init");
        double ref2 = read_scalar(rr, s);
        while (it < max_inner) {
          int st = run_cg(ow, MODE_APPLY, ip, nullptr, kappai, iq, nullptr, s);
          if (st) return st;
          check_hip(pcg_iteration(kpi, id, ir, iz, ip, iq, idinv, part, rz + (it & 1), rz + ((it + 1) & 1), rr,
                                  nullptr, n, s),
                    "pcg iteration");
          ++it;
          if (it % kCheckEvery != 0 && it != max_inner) continue;
          const double rr_now = read_scalar(rr, s);
          const bool finite = std::isfinite(rr_now);
          if (finite && rr_now > red2 * ref2 && rr_now > 0.25 * tol2 && it != max_inner) continue;
          // replacement: x += d (FP64), r = b - A64 x
          if (finite) check_hip(vec_axpy_f64(x, id, kpi, n, s), "axpy");
          rn2 = true_residual();
          ++outer;
          if (rn2 <= tol2) {
            status = TETMF_OK;
            break;
          }
          if (outer >= max_outer || it >= max_inner) break;
          const int keep = opi->prec == TETMF_F32 && finite && rn2 <= 4.0 * rr_now ? 1 : 0;
          check_hip(vec_cast(PREC_F64, r64, kpi, iq, n, s), "cast");
          check_hip(pcg_init(kpi, iq, idinv, id, ir, iz, ip, part, rz + (it & 1), rr, n, s, keep), "pcg restart");
          ref2 = read_scalar(rr, s);
        }
      }
      inner_total = it;
    }
    // iterative refinement (and the plain FP64 PCG: one outer step)
    for (; !(opi && opts->method == 1); ++outer) {
      const double rn2 = true_residual();
      if (rn2 <= tol2) {
        status = TETMF_OK;
        break;
      }
      if (outer >= max_outer) break;
      double target;
      const void* rhs;
      if (opi) {
        check_hip(vec_cast(PREC_F64, r64, kpi, iq, n, s), "cast");
        rhs = iq;
        target = opts->inner_rtol * opts->inner_rtol * rn2;
      } else {
        rhs = r64;
        target = 0.25 * tol2;
      }
      void* qscratch = opi ? (void*)tmp64 : iq;
      const int its = pcg(ow, opi ? kappai : kappa64, rhs, id, ir, iz, ip, qscratch, idinv, scal, part, target,
                          opts->max_inner, s);
      inner_total += its;
      check_hip(vec_axpy_f64(x, id, kpi, n, s), "axpy");
    }
    check_hip(hipStreamSynchronize(s), "sync");
    if (stats) {
      stats->outer_its = outer;
      stats->inner_its = inner_total;
      stats->final_relres = relres;
      stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (status != TETMF_OK) g_last_error = "tetmf_solve: iteration caps reached";
    return status;
  });
}

extern "C" int tetmf_chebyshev(tetmf_op* op, const void* kappa, const void* inv_diag, const void* b, void* x,
                               int degree, double lambda_min, double lambda_max, int zero_guess, void* stream) {
  return guarded([&]() -> int {
    if (!op || !inv_diag || !b || !x) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_chebyshev: NULL argument");
    if (op->kind != TETMF_CG) return fail(TETMF_ERR_UNSUPPORTED, "tetmf_chebyshev: only CG operators");
    if (degree < 1 || !std::isfinite(lambda_min) || !std::isfinite(lambda_max) || lambda_min < 0 ||
        !(lambda_min < lambda_max))
      return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_chebyshev: need degree >= 1 and 0 <= lambda_min < lambda_max");
    if (x == b || x == inv_diag) return fail(TETMF_ERR_ALIAS, "tetmf_chebyshev: x aliases b or inv_diag");
    DeviceScope dsc(op->device);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = op->nvec();
    if (op->cheb_bufs.empty()) {
      for (int i = 0; i < 2; ++i) {
        void* p = nullptr;
        check_hip(hipMalloc(&p, std::max<size_t>((size_t)n * op->esize(), 16)), "hipMalloc");
        op->cheb_bufs.push_back({p, (size_t)n * op->esize()});
      }
    }
    void* d = op->cheb_bufs[0].p;
    void* ax = op->cheb_bufs[1].p;
    const int kp = kernel_prec(op);
    const double theta = 0.5 * (lambda_max + lambda_min), delta = 0.5 * (lambda_max - lambda_min);
    if (zero_guess) {
      check_hip(cheb_step(kp, b, nullptr, inv_diag, d, x, 0.0, 1.0 / theta, 0, 0, n, s), "chebyshev step");
    } else {
      int st = run_cg(op, MODE_APPLY, x, nullptr, kappa, ax, nullptr, s);
      if (st) return st;
      check_hip(cheb_step(kp, b, ax, inv_diag, d, x, 0.0, 1.0 / theta, 0, 1, n, s), "chebyshev step");
    }
    double rho_prev = delta / theta;
    for (int k = 1; k < degree; ++k) {
      int st = run_cg(op, MODE_APPLY, x, nullptr, kappa, ax, nullptr, s);
      if (st) return st;
      const double rho = 1.0 / (2.0 * theta / delta - rho_prev);
      check_hip(cheb_step(kp, b, ax, inv_diag, d, x, rho * rho_prev, 2.0 * rho / delta, 1, 1, n, s),
                "chebyshev step");
      rho_prev = rho;
    }
    return TETMF_OK;
  });
}

namespace {

// Number of eigenvalues below t of the symmetric tridiagonal matrix (diag a,
// off-diagonal b) by the Sturm sequence of its LDL^T pivots.
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double t) {
  int count = 0;
  double q = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double off = i == 0 ? 0.0 : b[i - 1] * b[i - 1];
    q = a[i] - t - (i == 0 ? 0.0 : off / q);
    if (q == 0.0) q = -1e-300;
    if (q < 0) ++count;
  }
  return count;
}

double tridiag_lambda_max(const std::vector<double>& a, const std::vector<double>& b) {
  double lo = a[0], hi = a[0];
  for (size_t i = 0; i < a.size(); ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < a.size() ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  const int k = (int)a.size();
  for (int it = 0; it < 200 && hi - lo > 1e-14 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(a, b, mid) < k)
      lo = mid;  // the largest eigenvalue is above mid
    else
      hi = mid;
  }
  return hi;
}

}  // namespace

extern "C" int tetmf_estimate_lambda_max(tetmf_op* op, const void* kappa, const void* inv_diag, int n_iter,
                                         double* lambda_max, void* stream) {
  return guarded([&]() -> int {
    if (!op || !inv_diag || !lambda_max)
      return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_estimate_lambda_max: NULL argument");
    if (op->kind != TETMF_CG) return fail(TETMF_ERR_UNSUPPORTED, "tetmf_estimate_lambda_max: only CG operators");
    if (n_iter < 1 || n_iter > 500)
      return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_estimate_lambda_max: n_iter must be in 1..500");
    DeviceScope dsc(op->device);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = op->nvec();
    const size_t vb = std::max<size_t>((size_t)n * op->esize(), 16);
    // temporaries, freed on every exit path
    struct Tmp {
      std::vector<void*> v;
      ~Tmp() {
        for (void* p : v) (void)hipFree(p);
      }
    } tmp;
    auto al = [&](size_t bytes) {
      void* p = nullptr;
      check_hip(hipMalloc(&p, bytes), "hipMalloc");
      tmp.v.push_back(p);
      return p;
    };
    void* rhs = al(vb);
    void* xv = al(vb);
    void* r = al(vb);
    void* z = al(vb);
    void* pv = al(vb);
    void* q = al(vb);
    double* scal = (double*)al(8 * sizeof(double));
    double* part = (double*)al(3 * 512 * sizeof(double));
    const int kp = kernel_prec(op);
    check_hip(vec_hash_fill(kp, rhs, n, s), "fill");
    check_hip(pcg_init(kp, rhs, inv_diag, xv, r, z, pv, part, scal + 0, scal + 2, n, s), "pcg init");
    double rz_old = read_scalar(scal + 0, s);
    std::vector<double> alpha, beta;
    for (int it = 0; it < n_iter && rz_old > 0 && std::isfinite(rz_old); ++it) {
      int st = run_cg(op, MODE_APPLY, pv, nullptr, kappa, q, nullptr, s);
      if (st) return st;
      check_hip(pcg_iteration(kp, xv, r, z, pv, q, inv_diag, part, scal + (it & 1), scal + ((it + 1) & 1), scal + 2,
                              scal + 3, n, s),
                "pcg iteration");
      const double pq = read_scalar(scal + 3, s);
      const double rz_new = read_scalar(scal + ((it + 1) & 1), s);
      if (!(pq > 0) || !std::isfinite(pq)) break;
      alpha.push_back(rz_old / pq);
      beta.push_back(rz_new / rz_old);
      rz_old = rz_new;
    }
    check_hip(hipStreamSynchronize(s), "sync");
    if (alpha.empty()) return fail(TETMF_ERR_DEVICE, "tetmf_estimate_lambda_max: no conjugate-gradient step");
    // Lanczos tridiagonal matrix of D^-1 A from the conjugate-gradient coefficients
    const size_t k = alpha.size();
    std::vector<double> a(k), b(k > 0 ? k - 1 : 0);
    for (size_t j = 0; j < k; ++j) {
      a[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
      if (j + 1 < k) b[j] = std::sqrt(beta[j]) / alpha[j];
    }
    *lambda_max = tridiag_lambda_max(a, b);
    return TETMF_OK;
  });
}

extern "C" int tetmf_op_profile(tetmf_op* op, int enable) {
  return guarded([&]() -> int {
    if (!op) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_op_profile: NULL op");
    if (enable) op->events_used = 0;
    op->profiling = enable != 0;
    return TETMF_OK;
  });
}

extern "C" int tetmf_op_profile_read(tetmf_op* op, double* total_ms, int64_t* launches) {
  return guarded([&]() -> int {
    if (!op || !total_ms || !launches) return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_op_profile_read: NULL argument");
    DeviceScope ds(op->device);
    double sum = 0;
    for (size_t i = 0; i < op->events_used; ++i) {
      check_hip(hipEventSynchronize(op->events[2 * i + 1]), "hipEventSynchronize");
      float ms = 0;
      check_hip(hipEventElapsedTime(&ms, op->events[2 * i], op->events[2 * i + 1]), "hipEventElapsedTime");
      sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)op->events_used;
    return TETMF_OK;
  });
}
extern "C" int tetmf_op_profile_times(tetmf_op* op, double* ms, int64_t capacity, int64_t* launches) {
  return guarded([&]() -> int {
    if (!op || !ms || !launches || capacity < 0)
      return fail(TETMF_ERR_INVALID_ARGUMENT, "tetmf_op_profile_times: NULL argument or negative capacity");
    DeviceScope ds(op->device);
    const int64_t n = std::min<int64_t>((int64_t)op->events_used, capacity);
    for (int64_t i = 0; i < n; ++i) {
      check_hip(hipEventSynchronize(op->events[2 * i + 1]), "hipEventSynchronize");
      float t = 0;
      check_hip(hipEventElapsedTime(&t, op->events[2 * i], op->events[2 * i + 1]), "hipEventElapsedTime");
      ms[i] = t;
    }
    *launches = (int64_t)op->events_used;
    return TETMF_OK;
  });
}

extern "C" const char* tetmf_status_string(int status) {
  switch (status) {
    case TETMF_OK: return "ok";
    case TETMF_NOT_CONVERGED: return "not converged";
    case TETMF_ERR_INVALID_ARGUMENT: return "invalid argument";
    case TETMF_ERR_DEGENERATE_CELL: return "degenerate cell";
    case TETMF_ERR_NONCONFORMING_MESH: return "non-conforming mesh";
    case TETMF_ERR_UNSUPPORTED: return "unsupported";
    case TETMF_ERR_ALIAS: return "aliasing arguments";
    case TETMF_ERR_OUT_OF_MEMORY: return "out of memory";
    case TETMF_ERR_DEVICE: return "device error";
    default: return "unknown status";
  }
}

extern "C" const char* tetmf_last_error(void) { return g_last_error.c_str(); }
