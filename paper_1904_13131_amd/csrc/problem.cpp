// Host orchestration of the mfh library: levels, workspace layout,
// set_deformation, operator application, V-cycle, CG, Newton, and the C ABI.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "mfh.h"
#include "ops.hpp"
#include "tables.hpp"
#include "tuned.hpp"
#include "fused.hpp"
#include "vec.hpp"

namespace mfh {

const OpFns* op_fns(int dim, int degree) {
  if (dim == 2) {
    switch (degree) {
      case 1: return op_fns_2_1();
      case 2: return op_fns_2_2();
      case 3: return op_fns_2_3();
      case 4: return op_fns_2_4();
    }
  } else if (dim == 3) {
    switch (degree) {
      case 1: return op_fns_3_1();
      case 2: return op_fns_3_2();
      case 3: return op_fns_3_3();
      case 4: return op_fns_3_4();
    }
  }
  return nullptr;
}

struct Error : std::runtime_error {
  mfh_status st;
  Error(mfh_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

#define HIPCHECK(expr)                                                                        \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess)                                                                     \
      throw Error(MFH_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));           \
  } while (0)

static void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error(MFH_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Bump allocator over the caller's workspace; with base == nullptr it only measures.
struct Bump {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T) + 8;   // +8: never hand out zero-size slots at the same address
    return p;
  }
};

struct DevBand {
  int nout = 0, nin = 0, K = 0;
  int* start = nullptr;
  double* v64 = nullptr;
  float* v32 = nullptr;
  BandHost host;
  template <typename T>
  Band<T> get() const;
};
template <>
Band<double> DevBand::get<double>() const { return {nout, nin, K, start, v64}; }
template <>
Band<float> DevBand::get<float>() const { return {nout, nin, K, start, v32}; }

struct Level {
  int N = 0, L = 0;
  long long nn = 0, ndofs = 0, ncells = 0;
  long long csr_nnz = -1;      // nonzeros of the level's CSR pattern (computed on first request)
  double h = 0;
  Lattice lt{};
  int nwords = 0;
  uint32_t* bits = nullptr;
  double* u64 = nullptr;
  float* u32 = nullptr;
  double* cache64 = nullptr;
  float* cache32 = nullptr;
  double* diag64 = nullptr;
  void* dinv = nullptr;        // vcycle dtype
  void *vb = nullptr, *vx = nullptr, *vt = nullptr, *vd = nullptr;   // vcycle dtype
  double lam_max = 0;
  double lam_min = 0;          // coarsest level with the Chebyshev coarse solver
  double fix_max = 0, fix_min = 0;   // caller-fixed estimates (0: use the Lanczos ones)
  std::vector<double> cd, cr;  // Chebyshev step coefficients
  DevBand P1, R1, I1;          // transfers from level-1 into this level (l >= 1)
};

}  // namespace mfh

struct mfh_problem {
  mfh_desc d{};
  std::vector<double> mu, lam, mu2, incl;
  hipStream_t stream = nullptr;
  const mfh::OpFns* ops = nullptr;
  mfh::Tables<double> tb64{};
  mfh::Tables<float> tb32{};
  std::vector<mfh::Level> lv;
  int nq = 0;                        // quadrature points per cell
  // shared buffers
  double* incl_dev = nullptr;
  double* sc = nullptr;              // device scalars
  double* part = nullptr;            // reduction partials
  double* minj = nullptr;            // per level min J
  double* hist = nullptr;            // Lanczos alpha/beta history (2 * eig_iters per level)
  char* tmpA = nullptr;
  char* tmpB = nullptr;
  double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_Ap = nullptr;
  double *nw_R = nullptr, *nw_dg = nullptr, *nw_b = nullptr, *nw_du = nullptr, *nw_save = nullptr;
  double *f_ext = nullptr, *g1 = nullptr;   // dead-traction forces (finest level), 1-D lattice integrals
  // coarse level
  long long nf = 0;
  int* fmap = nullptr;               // dof -> free index or -1
  int* dof_of = nullptr;             // free index -> dof
  int* dof_perm = nullptr;           // position in the pivoted coarse inverse -> dof
  int* gj_sw = nullptr;              // exchange pairs of a block step
  double* Kinv = nullptr;
  double* Kc = nullptr;              // the assembled coarse tangent (kept for the inverse's acceptance test)
  double *gj_P = nullptr, *gj_C = nullptr, *gj_R = nullptr, *crf = nullptr, *czf = nullptr;
  int* flag = nullptr;
  double* elem = nullptr;            // element buffer of the ELEMENT scatter (finest level size)
  // FP64 work vectors of the Chebyshev coarse solver (coarse level size): 1/diag, b, x, t, d
  double *cc_dinv = nullptr, *cc_b = nullptr, *cc_x = nullptr, *cc_t = nullptr, *cc_d = nullptr;
  std::vector<int> h_fmap, h_dof_of;
  bool deformed = false;
  bool precond_ready = false;        // diagonals, lambda_max, coarse inverse built
  bool eig_ready = false;            // eigenvalue estimates exist (reused when eig_refresh allows)
  bool eig_fresh = false;            // this set-up recomputes them
  long long n_linearisations = 0;    // successful set_deformation calls
  bool has_coarse = false;           // coarse level small enough for the dense direct solve
  int coarse_negative = 0;           // negative pivots (eigenvalues) of the coarse tangent
  std::string err;
  // kernel timers
  bool timing = false;
  std::vector<hipEvent_t> ev;        // pairs (start, stop)
  size_t ev_used = 0;
  // V-cycle graph (captured on the problem's stream, replayed by the CG)
  bool use_graphs = false;
  bool graph_ready = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    graph_ready = false;
  }
  ~mfh_problem() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    drop_graph();
  }
};

namespace mfh {

namespace {

thread_local std::string g_err;

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

void validate(const mfh_desc* d) {
  auto bad = [](const std::string& m) { throw Error(MFH_ERR_INVALID_ARG, m); };
  if (!d) bad("descriptor is NULL");
  if (d->dim != 2 && d->dim != 3) bad("dim must be 2 or 3");
  if (d->degree < 1 || d->degree > kMaxDeg) bad("degree must be 1..4");
  if (d->n_cells < 1) bad("n_cells must be >= 1");
  // 32-bit lattice indexing: L = degree * n_cells + 1 with L^3 < 2^32, cells < 2^31
  if ((long long)d->degree * d->n_cells + 1 > 1600) bad("degree * n_cells + 1 must be <= 1600");
  if (d->n_levels < 1 || d->n_levels > 12) bad("n_levels must be 1..12");
  if (d->n_cells % (1 << (d->n_levels - 1)) != 0) bad("n_cells must be divisible by 2^(n_levels-1)");
  if (d->n_materials < 1 || d->n_materials > 2) bad("n_materials must be 1 or 2");
  if (!d->mu || !d->lambda) bad("mu/lambda arrays are NULL");
  for (int m = 0; m < d->n_materials; ++m)
    if (!(d->mu[m] > 0) || !std::isfinite(d->lambda[m])) bad("material parameters must have mu > 0 and finite lambda");
  if (d->n_inclusions < 0 || (d->n_inclusions > 0 && !d->inclusions)) bad("inclusions array is NULL");
  for (int s = 0; s < d->n_inclusions; ++s) {
    const double id = d->inclusions[s * (d->dim + 2) + d->dim + 1];
    if (id != 0.0 && (id != 1.0 || d->n_materials < 2)) bad("inclusion material id must be 0 or 1 (< n_materials)");
  }
  if (d->dirichlet_mask >> (2 * d->dim * d->dim)) bad("dirichlet_mask has bits beyond 2*dim*dim");
  if (d->qp_policy < 0 || d->qp_policy > 3) bad("qp_policy must be 0..3");
  if (d->law != MFH_LAW_NEO_HOOKE && d->law != MFH_LAW_MOONEY_RIVLIN) bad("bad law");
  if (d->law == MFH_LAW_MOONEY_RIVLIN) {
    if (d->qp_policy != MFH_QP_CACHE_T4) bad("the Mooney-Rivlin law needs qp_policy CACHE_T4");
    if (!d->mu2) bad("mu2 array is NULL");
    for (int m = 0; m < d->n_materials; ++m)
      if (!(d->mu2[m] >= 0) || !std::isfinite(d->mu2[m])) bad("mu2 must be finite and >= 0");
  }
  if (d->scatter < MFH_SCATTER_AUTO || d->scatter > MFH_SCATTER_ELEMENT) bad("bad scatter mode");
  if (d->tile_shape < MFH_TILE_SHAPE_AUTO || d->tile_shape > 1) bad("bad tile shape");
  if (d->cell_block < MFH_CELL_BLOCK_AUTO || d->cell_block > 1) bad("bad cell block");
  if (d->vcycle_dtype != MFH_F32 && d->vcycle_dtype != MFH_F64) bad("bad vcycle_dtype");
  if (d->cheb_degree < 1 || d->cheb_degree > 16) bad("cheb_degree must be 1..16");
  if (d->n_smooth < 1 || d->n_smooth > 8) bad("n_smooth must be 1..8");
  if (d->eig_iters < 1 || d->eig_iters > 200) bad("eig_iters must be 1..200");
  if (!(d->cheb_lo > 0) || !(d->cheb_hi > d->cheb_lo)) bad("need 0 < cheb_lo < cheb_hi");
  if (d->level_field != MFH_LEVEL_FIELD_NODAL && d->level_field != MFH_LEVEL_FIELD_VERTEX) bad("bad level_field");
  if (d->coarse_solver != MFH_COARSE_DIRECT && d->coarse_solver != MFH_COARSE_CHEBYSHEV) bad("bad coarse_solver");
  if (d->eig_refresh < 0) bad("eig_refresh must be >= 0");
}

// Largest coarse level that gets the dense FP64 direct solve; problems with a
// larger coarsest level support operator application but no V-cycle / CG.
constexpr long long kMaxCoarseDofs = 20000;
static_assert(kMaxCoarseDofs <= kGJMaxFree, "the pivoted coarse inverse holds at most kGJMaxFree free DoFs");
constexpr double kSingularTol = 1e-12;   // |pivot| <= kSingularTol * max |A_ii|: numerically singular

// Host-side level geometry, transfer tables and coarse-level maps.
void build_host(mfh_problem* P) {
  const mfh_desc& d = P->d;
  P->ops = op_fns(d.dim, d.degree);
  if (!P->ops) throw Error(MFH_ERR_INVALID_ARG, "no kernels for this (dim, degree)");
  P->tb64 = make_tables(d.degree);
  P->tb32 = to_float(P->tb64);
  const int n1 = d.degree + 1;
  P->nq = d.dim == 3 ? n1 * n1 * n1 : n1 * n1;
  P->lv.assign(d.n_levels, Level());
  for (int l = 0; l < d.n_levels; ++l) {
    Level& v = P->lv[l];
    v.N = d.n_cells >> (d.n_levels - 1 - l);
    v.L = d.degree * v.N + 1;
    v.nn = d.dim == 3 ? (long long)v.L * v.L * v.L : (long long)v.L * v.L;
    v.ndofs = d.dim * v.nn;
    v.ncells = d.dim == 3 ? (long long)v.N * v.N * v.N : (long long)v.N * v.N;
    v.h = 1.0 / v.N;
    v.nwords = (P->nq + 31) / 32;
    v.lt.L = v.L;
    v.lt.dim = d.dim;
    v.lt.nn = v.nn;
    for (int c = 0; c < 3; ++c) {
      unsigned fm = 0;
      if (c < d.dim)
        for (int f = 0; f < 2 * d.dim; ++f)
          if ((d.dirichlet_mask >> (f * d.dim + c)) & 1u) fm |= 1u << f;
      v.lt.fmask[c] = fm;
    }
    if (l >= 1) {
      const Level& c = P->lv[l - 1];
      const std::vector<double> Xf = lattice_coords(v.N, d.degree);
      const std::vector<double> Xc = lattice_coords(c.N, d.degree);
      const std::vector<double> P1 = eval_global_1d(c.N, d.degree, Xf);   // Lf x Lc
      std::vector<double> R1((size_t)c.L * v.L);
      for (int i = 0; i < v.L; ++i)
        for (int j = 0; j < c.L; ++j) R1[(size_t)j * v.L + i] = P1[(size_t)i * c.L + j];
      std::vector<double> I1;   // Lc x Lf: level displacement from this level to the coarser one
      if (d.level_field == MFH_LEVEL_FIELD_NODAL) {
        I1 = eval_global_1d(v.N, d.degree, Xc);
      } else {   // values at the coarse cell's vertices (fine nodes 2pe, 2p(e+1)), linear in between
        I1.assign((size_t)c.L * v.L, 0.0);
        const double hc = 1.0 / c.N;
        for (int J = 0; J < c.L; ++J) {
          const int e = std::min(J / d.degree, c.N - 1);
          const double t = (Xc[J] - e * hc) / hc;
          I1[(size_t)J * v.L + 2 * d.degree * e] += 1.0 - t;
          I1[(size_t)J * v.L + 2 * d.degree * (e + 1)] += t;
        }
      }
      v.P1.host = make_band(P1, v.L, c.L);
      v.R1.host = make_band(R1, c.L, v.L);
      v.I1.host = make_band(I1, c.L, v.L);
      for (DevBand* b : {&v.P1, &v.R1, &v.I1}) {
        b->nout = b->host.nout;
        b->nin = b->host.nin;
        b->K = b->host.K;
      }
    }
  }
  // coarse-level free DoFs
  Level& c = P->lv[0];
  P->h_fmap.assign(c.ndofs, -1);
  P->h_dof_of.clear();
  const bool direct = d.coarse_solver == MFH_COARSE_DIRECT;
  P->has_coarse = !direct || c.ndofs <= kMaxCoarseDofs;   // the Chebyshev coarse solver has no size limit
  for (long long dof = 0; direct && P->has_coarse && dof < c.ndofs; ++dof) {
    const int comp = (int)(dof / c.nn);
    long long n = dof - comp * c.nn;
    const int i = (int)(n % c.L);
    n /= c.L;
    const int j = (int)(n % c.L);
    const int k = (int)(n / c.L);
    unsigned f = 0;
    f |= (i == 0) ? 1u : 0u;
    f |= (i == c.L - 1) ? 2u : 0u;
    f |= (j == 0) ? 4u : 0u;
    f |= (j == c.L - 1) ? 8u : 0u;
    if (d.dim == 3) {
      f |= (k == 0) ? 16u : 0u;
      f |= (k == c.L - 1) ? 32u : 0u;
    }
    if (!(f & c.lt.fmask[comp])) {
      P->h_fmap[dof] = (int)P->h_dof_of.size();
      P->h_dof_of.push_back((int)dof);
    }
  }
  P->nf = (long long)P->h_dof_of.size();
}

// Assigns every device buffer; returns the bytes used.
// Scatter of the tangent vmult on level v in precision t (0: FP64, 1: FP32):
// the descriptor's mode, or with MFH_SCATTER_AUTO the measured choice for
// (dim, degree, precision, qp policy, cells of the level).
int scatter_mode(const mfh_problem* P, const Level& v, int t) {
  if (P->d.scatter != MFH_SCATTER_AUTO) return P->d.scatter;
  return tuned_scatter(P->d.dim, P->d.degree, t, P->d.qp_policy, v.ncells);
}

// Tile shape of the TILE scatter on a level: the descriptor's, or with
// MFH_TILE_SHAPE_AUTO the faster of the two measured for the level.
int tile_shape(const mfh_problem* P, const Level& v, int t) {
  if (P->d.tile_shape != MFH_TILE_SHAPE_AUTO) return P->d.tile_shape;
  return tuned_tile(P->d.dim, P->d.degree, t, P->d.qp_policy, v.ncells);
}

// Cell-block variant of the tangent vmult's pencil kernels on a level: the
// descriptor's, or with MFH_CELL_BLOCK_AUTO the tuned one.
int cell_block(const mfh_problem* P, const Level& v, int t) {
  if (P->d.cell_block != MFH_CELL_BLOCK_AUTO) return P->d.cell_block;
  return tuned_cell_block(P->d.dim, P->d.degree, t, P->d.qp_policy, v.ncells);
}

size_t layout(mfh_problem* P, char* base) {
  const mfh_desc& d = P->d;
  Bump b;
  b.base = base;
  const size_t vs = d.vcycle_dtype == MFH_F32 ? sizeof(float) : sizeof(double);
  const int nw = P->ops->cache_words[d.qp_policy];
  for (size_t l = 0; l < P->lv.size(); ++l) {
    Level& v = P->lv[l];
    v.bits = b.take<uint32_t>((size_t)v.ncells * v.nwords);
    v.u64 = b.take<double>(v.ndofs);
    v.u32 = b.take<float>(v.ndofs);
    v.cache64 = nw ? b.take<double>((size_t)nw * P->nq * v.ncells) : nullptr;
    v.cache32 = nw ? b.take<float>((size_t)nw * P->nq * v.ncells) : nullptr;
    v.diag64 = b.take<double>(v.ndofs);
    v.dinv = b.take<char>(vs * v.ndofs);
    v.vb = b.take<char>(vs * v.ndofs);
    v.vx = b.take<char>(vs * v.ndofs);
    v.vt = b.take<char>(vs * v.ndofs);
    v.vd = b.take<char>(vs * v.ndofs);
    for (DevBand* db : {&v.P1, &v.R1, &v.I1}) {
      if (!db->nout) continue;
      db->start = b.take<int>(db->nout);
      db->v64 = b.take<double>((size_t)db->nout * db->K);
      db->v32 = b.take<float>((size_t)db->nout * db->K);
    }
  }
  const Level& top = P->lv.back();
  P->incl_dev = b.take<double>((size_t)std::max(1, d.n_inclusions) * (d.dim + 2));
  P->sc = b.take<double>(SC_COUNT);
  P->part = b.take<double>((size_t)std::max<long long>(kRedBlocks, top.ncells / P->ops->cpb[0] + 16));
  P->minj = b.take<double>(P->lv.size());
  P->hist = b.take<double>(2 * (size_t)d.eig_iters * P->lv.size() + 2);
  // transfer intermediates: dim * Lf^(dim-1) * Lc entries of up to 8 bytes
  size_t tmp = 8;
  for (size_t l = 1; l < P->lv.size(); ++l) {
    const size_t Lf = P->lv[l].L, Lc = P->lv[l - 1].L;
    const size_t sz = d.dim * (d.dim == 3 ? Lf * Lf * Lc : Lf * Lc);
    tmp = std::max(tmp, sz);
  }
  P->tmpA = b.take<char>(tmp * 8);
  P->tmpB = b.take<char>(tmp * 8);
  P->cg_r = b.take<double>(top.ndofs);
  P->cg_z = b.take<double>(top.ndofs);
  P->cg_p = b.take<double>(top.ndofs);
  P->cg_Ap = b.take<double>(top.ndofs);
  P->nw_R = b.take<double>(top.ndofs);
  P->nw_dg = b.take<double>(top.ndofs);
  P->nw_b = b.take<double>(top.ndofs);
  P->nw_du = b.take<double>(top.ndofs);
  P->nw_save = b.take<double>(top.ndofs);
  P->f_ext = b.take<double>(top.ndofs);
  P->g1 = b.take<double>(top.L);
  const Level& c = P->lv[0];
  P->fmap = b.take<int>(P->has_coarse ? c.ndofs : 1);
  P->dof_of = b.take<int>(std::max<long long>(1, P->nf));
  P->dof_perm = b.take<int>(std::max<long long>(1, P->nf));
  P->gj_sw = b.take<int>(1 + 4 * 64);
  P->Kinv = b.take<double>((size_t)P->nf * P->nf);
  P->Kc = b.take<double>((size_t)P->nf * P->nf);
  P->gj_P = b.take<double>(64 * 64);
  P->gj_C = b.take<double>((size_t)P->nf * 64);
  P->gj_R = b.take<double>((size_t)P->nf * 64);
  P->crf = b.take<double>(std::max<long long>(1, P->nf));
  P->czf = b.take<double>(std::max<long long>(1, P->nf));
  P->flag = b.take<int>(3);
  if (d.coarse_solver == MFH_COARSE_CHEBYSHEV) {
    const long long n0 = P->lv[0].ndofs;
    for (double** q : {&P->cc_dinv, &P->cc_b, &P->cc_x, &P->cc_t, &P->cc_d}) *q = b.take<double>(n0);
  }
  size_t nodes_per_cell = 1;
  for (int k = 0; k < d.dim; ++k) nodes_per_cell *= (size_t)(d.degree + 1);
  bool any_elem = false;
  for (const Level& v : P->lv)
    for (int t = 0; t < 2; ++t) any_elem |= scatter_mode(P, v, t) == MFH_SCATTER_ELEMENT;
  P->elem = any_elem ? b.take<double>((size_t)d.dim * nodes_per_cell * top.ncells) : nullptr;
  return b.off + 256;
}

template <typename T>
CellArgs<T> cell_args(const mfh_problem* P, const Level& v, const T* u, const T* cache, const T* x, T* y);

template <typename T>
void fill_common(const mfh_problem* P, const Level& v, CellArgs<T>& a) {
  a.N = v.N;
  a.L = v.L;
  a.nn = v.nn;
  a.ncells = v.ncells;
  a.nlaunch = v.ncells;
  a.color = -1;
  for (int c = 0; c < 3; ++c) a.fmask[c] = v.lt.fmask[c];
  a.invh = (T)(1.0 / v.h);
  a.wscale = (T)std::pow(v.h, P->d.dim - 1);
  for (int m = 0; m < 2; ++m) {
    const int mm = m < P->d.n_materials ? m : 0;
    a.mu[m] = (T)P->mu[mm];
    a.lam[m] = (T)P->lam[mm];
    a.mu2[m] = (T)P->mu2[mm];
  }
  a.law = P->d.law == MFH_LAW_MOONEY_RIVLIN ? 1 : 0;
  a.matbits = v.bits;
  a.nwords = v.nwords;
  a.blockmin = P->part;
  a.mask_in = 1;
}

template <>
CellArgs<double> cell_args<double>(const mfh_problem* P, const Level& v, const double* u, const double* cache,
                                   const double* x, double* y) {
  CellArgs<double> a{};
  a.tb = P->tb64;
  fill_common(P, v, a);
  a.u = u;
  a.cache = cache;
  a.x = x;
  a.y = y;
  return a;
}
template <>
CellArgs<float> cell_args<float>(const mfh_problem* P, const Level& v, const float* u, const float* cache,
                                 const float* x, float* y) {
  CellArgs<float> a{};
  a.tb = P->tb32;
  fill_common(P, v, a);
  a.u = u;
  a.cache = cache;
  a.x = x;
  a.y = y;
  return a;
}

template <typename T>
struct Sel;
template <>
struct Sel<double> {
  static const double* u(const Level& v) { return v.u64; }
  static const double* cache(const Level& v) { return v.cache64; }
  static void run(const OpFns* o, int cb, int pol, const CellArgs<double>& a, unsigned g, hipStream_t s) {
    o->tangent_d[cb][pol](a, g, s);
  }
  static void run_tile(const OpFns* o, int shape, int pol, const CellArgs<double>& a, unsigned g, hipStream_t s) {
    o->tangent_tile_d[shape][pol](a, g, s);
  }
  static void elem_gather(const OpFns* o, int cb, const CellArgs<double>& a, hipStream_t s) {
    o->elem_gather_d[cb](a, s);
  }
  static void elem_gather_cheb(const OpFns* o, int cb, const CellArgs<double>& a, const ChebOut<double>& c,
                               hipStream_t s) {
    o->elem_gather_cheb_d[cb](a, c, s);
  }
  static Band<double> band(const DevBand& b) { return b.get<double>(); }
};
template <>
struct Sel<float> {
  static const float* u(const Level& v) { return v.u32; }
  static const float* cache(const Level& v) { return v.cache32; }
  static void run(const OpFns* o, int cb, int pol, const CellArgs<float>& a, unsigned g, hipStream_t s) {
    o->tangent_f[cb][pol](a, g, s);
  }
  static void run_tile(const OpFns* o, int shape, int pol, const CellArgs<float>& a, unsigned g, hipStream_t s) {
    o->tangent_tile_f[shape][pol](a, g, s);
  }
  static void elem_gather(const OpFns* o, int cb, const CellArgs<float>& a, hipStream_t s) {
    o->elem_gather_f[cb](a, s);
  }
  static void elem_gather_cheb(const OpFns* o, int cb, const CellArgs<float>& a, const ChebOut<float>& c,
                               hipStream_t s) {
    o->elem_gather_cheb_f[cb](a, c, s);
  }
  static Band<float> band(const DevBand& b) { return b.get<float>(); }
};

long long color_count(int N, int dim, int color) {
  long long c = 1;
  for (int ax = 0; ax < dim; ++ax) {
    const int bit = (color >> ax) & 1;
    c *= (N - bit + 1) / 2;
  }
  return c;
}

void timer_mark(mfh_problem* P) {
  if (!P->timing) return;
  if (P->ev_used == P->ev.size()) {
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    P->ev.push_back(e);
  }
  HIPCHECK(hipEventRecord(P->ev[P->ev_used++], P->stream));
}

// y = K_c x (mask_in = 1) or y = (I - C) K x with constrained rows zero (mask_in = 0).
template <typename T>
void vmult(mfh_problem* P, int l, const T* x, T* y, int mask_in = 1) {
  const Level& v = P->lv[l];
  CellArgs<T> a = cell_args<T>(P, v, Sel<T>::u(v), Sel<T>::cache(v), x, y);
  a.mask_in = mask_in;
  const int ti = std::is_same<T, double>::value ? 0 : 1;
  const int cb = cell_block(P, v, ti);
  const int cpb = P->ops->cpb[cb];
  const int mode = scatter_mode(P, v, ti);
  if (mode == MFH_SCATTER_ELEMENT) {   // cell kernel into the element buffer, then the node sums
    a.elem = reinterpret_cast<T*>(P->elem);
    timer_mark(P);
    Sel<T>::run(P->ops, cb, P->d.qp_policy, a, (unsigned)((v.ncells + cpb - 1) / cpb), P->stream);
    Sel<T>::elem_gather(P->ops, cb, a, P->stream);
    timer_mark(P);
    return;
  }
  fill_dirichlet<T>(y, mask_in ? x : nullptr, v.ndofs, v.lt, P->stream);
  timer_mark(P);
  if (mode == MFH_SCATTER_TILE) {
    const int ts = tile_shape(P, v, ti);
    Sel<T>::run_tile(P->ops, ts, P->d.qp_policy, a, (unsigned)P->ops->tiles[ti][ts](v.N), P->stream);
  } else if (mode == MFH_SCATTER_ATOMIC) {
    Sel<T>::run(P->ops, cb, P->d.qp_policy, a, (unsigned)((v.ncells + cpb - 1) / cpb), P->stream);
  } else {
    for (int color = 0; color < (1 << P->d.dim); ++color) {
      a.color = color;
      a.nlaunch = color_count(v.N, P->d.dim, color);
      if (!a.nlaunch) continue;
      Sel<T>::run(P->ops, cb, P->d.qp_policy, a, (unsigned)((a.nlaunch + cpb - 1) / cpb), P->stream);
    }
  }
  timer_mark(P);
}

// One Chebyshev step with its operator application, on a level whose vmult
// uses the ELEMENT scatter: the cell kernel writes the element buffer and the
// node-sum kernel applies the step to x and d directly (same arithmetic as
// vmult followed by cheb_step, without the product vector).  Returns false
// (nothing enqueued) on levels with another scatter.
template <typename T>
bool vmult_cheb(mfh_problem* P, int l, const T* f, const T* dinv, T* d, T* x, T cd, T cr) {
  const Level& v = P->lv[l];
  if (scatter_mode(P, v, std::is_same<T, double>::value ? 0 : 1) != MFH_SCATTER_ELEMENT) return false;
  CellArgs<T> a = cell_args<T>(P, v, Sel<T>::u(v), Sel<T>::cache(v), x, nullptr);
  a.mask_in = 1;
  a.elem = reinterpret_cast<T*>(P->elem);
  const int cb = cell_block(P, v, std::is_same<T, double>::value ? 0 : 1);
  const int cpb = P->ops->cpb[cb];
  timer_mark(P);
  Sel<T>::run(P->ops, cb, P->d.qp_policy, a, (unsigned)((v.ncells + cpb - 1) / cpb), P->stream);
  Sel<T>::elem_gather_cheb(P->ops, cb, a, ChebOut<T>{f, dinv, d, x, cd, cr}, P->stream);
  timer_mark(P);
  return true;
}

void residual(mfh_problem* P, const double* u, double* r) {
  const Level& v = P->lv.back();
  fill_dirichlet<double>(r, nullptr, v.ndofs, v.lt, P->stream);
  CellArgs<double> a = cell_args<double>(P, v, u, nullptr, nullptr, r);
  const int cpb = P->ops->cpb[0];
  if (P->d.scatter != MFH_SCATTER_COLOR) {
    P->ops->residual(a, (unsigned)((v.ncells + cpb - 1) / cpb), P->stream);
  } else {
    for (int color = 0; color < (1 << P->d.dim); ++color) {
      a.color = color;
      a.nlaunch = color_count(v.N, P->d.dim, color);
      if (!a.nlaunch) continue;
      P->ops->residual(a, (unsigned)((a.nlaunch + cpb - 1) / cpb), P->stream);
    }
  }
}

// Applies the three (two) 1-D sweeps of a tensor-product transfer.
template <typename T>
void transfer(mfh_problem* P, const DevBand& band, int Lin, int Lout, const T* in, T* out, bool add, bool mask,
              const Lattice& out_lt) {
  const int dim = P->d.dim;
  SweepArgs<T> a{};
  a.band = Sel<T>::band(band);
  a.comps = dim;
  a.add = 0;
  a.mask = 0;
  int n[3] = {Lin, Lin, dim == 3 ? Lin : 1};
  const T* src = in;
  T* bufs[2] = {reinterpret_cast<T*>(P->tmpA), reinterpret_cast<T*>(P->tmpB)};
  for (int ax = 0; ax < dim; ++ax) {
    const bool last = ax == dim - 1;
    a.axis = ax;
    a.n[0] = n[0];
    a.n[1] = n[1];
    a.n[2] = n[2];
    a.in_cs = (long long)n[0] * n[1] * n[2];
    int m[3] = {n[0], n[1], n[2]};
    m[ax] = Lout;
    a.out_cs = (long long)m[0] * m[1] * m[2];
    T* dst = last ? out : bufs[ax & 1];
    if (last) {
      a.add = add ? 1 : 0;
      a.mask = mask ? 1 : 0;
      a.lt = out_lt;
    }
    sweep<T>(src, dst, a, P->stream);
    src = dst;
    n[0] = m[0];
    n[1] = m[1];
    n[2] = m[2];
  }
}

template <typename T>
void prolongate(mfh_problem* P, int l, const T* xc, T* yf, bool add) {
  const Level& f = P->lv[l];
  const Level& c = P->lv[l - 1];
  transfer<T>(P, f.P1, c.L, f.L, xc, yf, add, true, f.lt);
}

template <typename T>
void restrict_(mfh_problem* P, int l, const T* xf, T* yc) {
  const Level& f = P->lv[l];
  const Level& c = P->lv[l - 1];
  transfer<T>(P, f.R1, f.L, c.L, xf, yc, false, true, c.lt);
}

// ---- smoother, V-cycle ---------------------------------------------------------------

template <typename T>
void cheb_apply(mfh_problem* P, int l, const T* f, T* x, bool xzero) {
  Level& v = P->lv[l];
  T* t = static_cast<T*>(v.vt);
  T* dvec = static_cast<T*>(v.vd);
  const T* dinv = static_cast<const T*>(v.dinv);
  for (int j = 0; j < (int)v.cd.size(); ++j) {
    const bool first_zero = (j == 0 && xzero);
    const T* tt = nullptr;
    if (!first_zero) {
      if (vmult_cheb<T>(P, l, f, dinv, dvec, x, (T)v.cd[j], (T)v.cr[j])) continue;
      vmult<T>(P, l, x, t);
      tt = t;
    }
    cheb_step<T>(f, tt, dinv, dvec, x, (T)v.cd[j], (T)v.cr[j], first_zero ? 1 : 0, v.ndofs, P->stream);
  }
}

template <typename T>
void smooth(mfh_problem* P, int l, const T* f, T* x, bool xzero) {
  for (int s = 0; s < P->d.n_smooth; ++s) cheb_apply<T>(P, l, f, x, xzero && s == 0);
}

template <typename T>
void coarse_solve(mfh_problem* P, const T* b, T* x) {
  const Level& c = P->lv[0];
  const long long n = c.ndofs;
  if (P->d.coarse_solver == MFH_COARSE_CHEBYSHEV) {   // FP64 Chebyshev iteration from x = 0
    cast<T, double>(b, P->cc_b, n, P->stream);
    for (int j = 0; j < (int)c.cd.size(); ++j) {
      const bool first = j == 0;
      if (!first) vmult<double>(P, 0, P->cc_x, P->cc_t);
      cheb_step<double>(P->cc_b, first ? nullptr : P->cc_t, P->cc_dinv, P->cc_d, P->cc_x, c.cd[j], c.cr[j],
                        first ? 1 : 0, n, P->stream);
    }
    cast<double, T>(P->cc_x, x, n, P->stream);
    return;
  }
  fill<T>(x, T(0), n, P->stream);
  if (P->nf) coarse_apply<T>(P->Kinv, P->nf, P->dof_perm, b, P->crf, P->czf, x, P->stream);
}

template <typename T>
void vcycle_level(mfh_problem* P, int l, const T* b, T* x) {
  if (l == 0) {
    coarse_solve<T>(P, b, x);
    return;
  }
  Level& v = P->lv[l];
  Level& c = P->lv[l - 1];
  T* t = static_cast<T*>(v.vt);
  smooth<T>(P, l, b, x, true);
  vmult<T>(P, l, x, t);
  lincomb3<T>(t, T(1), b, T(-1), t, T(0), nullptr, v.ndofs, P->stream);
  restrict_<T>(P, l, t, static_cast<T*>(c.vb));
  vcycle_level<T>(P, l - 1, static_cast<T*>(c.vb), static_cast<T*>(c.vx));
  prolongate<T>(P, l, static_cast<T*>(c.vx), x, true);
  smooth<T>(P, l, b, x, false);
}

void vcycle(mfh_problem* P, const double* r, double* z) {
  const int top = (int)P->lv.size() - 1;
  Level& v = P->lv[top];
  if (P->d.vcycle_dtype == MFH_F32) {
    cast<double, float>(r, static_cast<float*>(v.vb), v.ndofs, P->stream);
    vcycle_level<float>(P, top, static_cast<float*>(v.vb), static_cast<float*>(v.vx));
    cast<float, double>(static_cast<float*>(v.vx), z, v.ndofs, P->stream);
  } else {
    vcycle_level<double>(P, top, r, z);
  }
}

double read_scalar(mfh_problem* P, const double* dev) {
  double h = 0;
  HIPCHECK(hipMemcpyAsync(&h, dev, sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIPCHECK(hipStreamSynchronize(P->stream));
  return h;
}

// Largest eigenvalue of D^-1 A on level l from eig_iters Jacobi-PCG steps
// (CG-Lanczos relation), in the V-cycle precision.  The iterations are
// enqueued here; their alpha/beta history lands in hist (2 * eig_iters).
template <typename T>
void lanczos_enqueue(mfh_problem* P, int l, double* hist) {
  Level& v = P->lv[l];
  const long long n = v.ndofs;
  T* r = static_cast<T*>(v.vb);
  T* z = static_cast<T*>(v.vx);
  T* p = static_cast<T*>(v.vd);
  T* Ap = static_cast<T*>(v.vt);
  const T* dinv = static_cast<const T*>(v.dinv);
  splitmix_uniform<T>(r, n, 0x5EEDull, P->stream);
  zero_constrained<T>(r, n, v.lt, P->stream);
  cheb_step<T>(r, nullptr, dinv, z, p, T(0), T(1), 1, n, P->stream);   // z = D^-1 r, p = z
  dot<T, T>(r, z, n, P->part, P->sc + SC_RZ, P->stream);
  const int it = P->d.eig_iters;
  for (int j = 0; j < it; ++j) {
    vmult<T>(P, l, p, Ap);
    dot<T, T>(p, Ap, n, P->part, P->sc + SC_PAP, P->stream);
    scalar_div(P->sc, SC_ALPHA, SC_RZ, SC_PAP, -1, -1, hist, j, P->stream);
    lanczos_update<T>(r, z, Ap, dinv, n, P->sc, P->part, P->stream);
    scalar_div(P->sc, SC_BETA, SC_RZNEW, SC_RZ, SC_RZ, SC_RZNEW, hist, it + j, P->stream);
    cg_pupdate<T>(p, z, n, P->sc, P->stream);
  }
}

// The same estimate on the coarsest level in FP64 (Chebyshev coarse solver),
// on the solver's own FP64 vectors.
void coarse_lanczos_enqueue(mfh_problem* P, double* hist) {
  Level& v = P->lv[0];
  const long long n = v.ndofs;
  double *r = P->cc_b, *z = P->cc_x, *p = P->cc_d, *Ap = P->cc_t;
  splitmix_uniform<double>(r, n, 0x5EEDull, P->stream);
  zero_constrained<double>(r, n, v.lt, P->stream);
  cheb_step<double>(r, nullptr, P->cc_dinv, z, p, 0.0, 1.0, 1, n, P->stream);
  dot<double, double>(r, z, n, P->part, P->sc + SC_RZ, P->stream);
  const int it = P->d.eig_iters;
  for (int j = 0; j < it; ++j) {
    vmult<double>(P, 0, p, Ap);
    dot<double, double>(p, Ap, n, P->part, P->sc + SC_PAP, P->stream);
    scalar_div(P->sc, SC_ALPHA, SC_RZ, SC_PAP, -1, -1, hist, j, P->stream);
    lanczos_update<double>(r, z, Ap, P->cc_dinv, n, P->sc, P->part, P->stream);
    scalar_div(P->sc, SC_BETA, SC_RZNEW, SC_RZ, SC_RZ, SC_RZNEW, hist, it + j, P->stream);
    cg_pupdate<double>(p, z, n, P->sc, P->stream);
  }
}

// Host side of the estimate: the Lanczos tridiagonal from the CG coefficients
// (up to the first non-positive or non-finite one) and its largest eigenvalue.
double lanczos_lambda(const double* h, int it, int l, double* lam_min = nullptr) {
  std::vector<double> al, be;
  for (int j = 0; j < it; ++j) {
    const double a = h[j], bta = h[it + j];
    if (!(a > 0) || !std::isfinite(a)) break;
    al.push_back(a);
    be.push_back(bta);
    if (!(bta > 0) || !std::isfinite(bta)) break;
  }
  const int m = (int)al.size();
  if (m == 0) throw Error(MFH_ERR_BREAKDOWN, "eigenvalue estimate: CG broke down on level " + std::to_string(l));
  std::vector<double> dg(m), off(m > 1 ? m - 1 : 0);
  for (int j = 0; j < m; ++j) {
    dg[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
    if (j + 1 < m) off[j] = std::sqrt(be[j]) / al[j];
  }
  if (lam_min) *lam_min = tridiag_min_eig(dg, off);
  return tridiag_max_eig(dg, off);
}

// Coefficients of a degree-`degree` Chebyshev iteration on [lo, hi]
// (Saad, Alg. 12.1), applied by cheb_step.
void set_cheb_interval(Level& v, double lo, double hi, int degree) {
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  v.cd.assign(degree, 0.0);
  v.cr.assign(degree, 0.0);
  double rho = 1.0 / sigma;
  v.cr[0] = 1.0 / theta;
  for (int j = 1; j < degree; ++j) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    v.cd[j] = rn * rho;
    v.cr[j] = 2.0 * rn / delta;
    rho = rn;
  }
}

void set_cheb_coeffs(mfh_problem* P, Level& v) {
  set_cheb_interval(v, P->d.cheb_lo * v.lam_max, P->d.cheb_hi * v.lam_max, P->d.cheb_degree);
}

// Chebyshev iteration as the coarse solver (Sec. 7): on [lam_min, cheb_hi *
// lam_max], of the degree whose error bound 1 / T_k((b + a) / (b - a)) reaches
// 1e-3.
constexpr double kCoarseReduction = 1e-3;
void set_coarse_chebyshev(mfh_problem* P, Level& v) {
  if (!(v.lam_min > 0) || !(v.lam_max > v.lam_min))
    throw Error(MFH_ERR_NOT_SPD, "Chebyshev coarse solver: the coarse tangent is not definite (lambda_min estimate " +
                                     std::to_string(v.lam_min) + ")");
  const double a = v.lam_min, b = P->d.cheb_hi * v.lam_max;
  const double k = std::acosh(1.0 / kCoarseReduction) / std::acosh((b + a) / (b - a));
  const int degree = (int)std::min(1000.0, std::max(1.0, std::ceil(k)));
  set_cheb_interval(v, a, b, degree);
}

void interpolate_down(mfh_problem* P, int l) {
  const Level& f = P->lv[l];
  const Level& c = P->lv[l - 1];
  transfer<double>(P, f.I1, f.L, c.L, f.u64, c.u64, false, false, c.lt);
}

// External force of dead face tractions on the finest level (Sec. 3's Neumann
// term): the 1-D integrals of the global basis functions over [0, 1] are
// g[I] = sum over cells e holding node I of h sum_q w_q phi_(I - p e)(x_q);
// a face node's force is t_f times the product of g over the face's
// tangential axes.  Constrained rows are zeroed.
void external_force(mfh_problem* P, const double* ft, double* f) {
  const Level& v = P->lv.back();
  const int p = P->d.degree;
  std::vector<double> m1(p + 1, 0.0), g(v.L, 0.0);
  for (int b = 0; b <= p; ++b)
    for (int q = 0; q <= p; ++q) m1[b] += v.h * P->tb64.w[q] * P->tb64.S[q][b];
  for (int e = 0; e < v.N; ++e)
    for (int b = 0; b <= p; ++b) g[p * e + b] += m1[b];
  HIPCHECK(hipMemcpyAsync(P->g1, g.data(), sizeof(double) * v.L, hipMemcpyHostToDevice, P->stream));
  HIPCHECK(hipStreamSynchronize(P->stream));   // g goes out of scope
  traction_force(f, v.lt, ft, P->g1, v.ndofs, P->stream);
  zero_constrained<double>(f, v.ndofs, v.lt, P->stream);
  check_launch("external force");
}

// Builds every level operator about u (Sec. 6): enqueues the level
// displacements and quadrature data; min J of every level lands in P->minj.
void setdef_enqueue(mfh_problem* P, const double* u) {
  const mfh_desc& d = P->d;
  P->drop_graph();
  P->deformed = false;
  P->precond_ready = false;
  const int nl = (int)P->lv.size();
  hipStream_t s = P->stream;
  Level& top = P->lv.back();
  HIPCHECK(hipMemcpyAsync(top.u64, u, sizeof(double) * top.ndofs, hipMemcpyDeviceToDevice, s));
  for (int l = nl - 1; l >= 1; --l) interpolate_down(P, l);
  const int pol = d.qp_policy;
  const int cpb = P->ops->cpb[0];
  for (int l = 0; l < nl; ++l) {
    Level& v = P->lv[l];
    cast<double, float>(v.u64, v.u32, v.ndofs, s);
    CellArgs<double> a = cell_args<double>(P, v, v.u64, nullptr, nullptr, nullptr);
    const unsigned g = (unsigned)((v.ncells + cpb - 1) / cpb);
    P->ops->qpdata_d[pol](a, v.cache64, g, s);
    if (pol != MFH_QP_RECOMPUTE) P->ops->qpdata_f[pol](a, v.cache32, g, s);
    min_reduce(P->part, (int)g, P->minj + l, s);
  }
  check_launch("quadrature data");
}

// Host side after the stream has drained: min J over the levels (mj[nl]
// copied from P->minj); an inverted quadrature point is an error.
double setdef_finish(mfh_problem* P, const double* mj) {
  double minJ = 1e300;
  for (size_t l = 0; l < P->lv.size(); ++l) minJ = std::fmin(minJ, mj[l]);
  if (!(minJ > 0)) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "deformation inverts a quadrature point: min J = %.6g", minJ);
    throw Error(MFH_ERR_INVERTED, buf);
  }
  P->deformed = true;
  ++P->n_linearisations;
  return minJ;
}

double set_deformation(mfh_problem* P, const double* u) {
  setdef_enqueue(P, u);
  std::vector<double> mj(P->lv.size());
  HIPCHECK(hipMemcpyAsync(mj.data(), P->minj, sizeof(double) * mj.size(), hipMemcpyDeviceToHost, P->stream));
  HIPCHECK(hipStreamSynchronize(P->stream));
  return setdef_finish(P, mj.data());
}

// Preconditioner data about the current linearisation point: operator
// diagonals, Chebyshev intervals (lambda_max) and the coarse inverse.  Built on
// the first solver call after every set_deformation.  The enqueue half issues
// all device work; the host half needs the Lanczos histories (P->hist) and
// the coarse pivot flags (P->flag) copied back.
size_t setup_host_words(const mfh_problem* P) { return 2 * (size_t)P->d.eig_iters * P->lv.size() + 2; }

void setup_enqueue(mfh_problem* P) {
  const mfh_desc& d = P->d;
  const int nl = (int)P->lv.size();
  hipStream_t s = P->stream;
  for (int l = 0; l < nl; ++l) {
    Level& v = P->lv[l];
    fill<double>(v.diag64, 0.0, v.ndofs, s);
    CellArgs<double> a = cell_args<double>(P, v, v.u64, nullptr, nullptr, v.diag64);
    P->ops->diag(a, s);
    set_constrained<double>(v.diag64, 1.0, v.ndofs, v.lt, s);
    if (d.vcycle_dtype == MFH_F32)
      reciprocal<float>(v.diag64, static_cast<float*>(v.dinv), v.ndofs, s);
    else
      reciprocal<double>(v.diag64, static_cast<double*>(v.dinv), v.ndofs, s);
  }
  check_launch("diagonal");
  const int it = d.eig_iters;
  const bool cheb_coarse = d.coarse_solver == MFH_COARSE_CHEBYSHEV;
  // eigenvalue estimates: every eig_refresh-th linearisation (0: only the first)
  P->eig_fresh = !P->eig_ready ||
                 (d.eig_refresh > 0 && (P->n_linearisations - 1) % d.eig_refresh == 0);
  for (int l = 1; P->eig_fresh && l < nl; ++l) {
    double* h = P->hist + 2 * (size_t)it * l;
    if (d.vcycle_dtype == MFH_F32)
      lanczos_enqueue<float>(P, l, h);
    else
      lanczos_enqueue<double>(P, l, h);
  }
  if (cheb_coarse) {   // the coarse solver runs in FP64 whatever the V-cycle precision
    reciprocal<double>(P->lv[0].diag64, P->cc_dinv, P->lv[0].ndofs, s);
    if (P->eig_fresh) coarse_lanczos_enqueue(P, P->hist);
  }
  // coarse level (direct solver): dense FP64 tangent on free DoFs and its inverse
  // (kept in the pivoted basis when the pivoted pass runs; dof_perm maps it)
  Level& c = P->lv[0];
  const long long nf = P->nf;
  fill<int>(P->flag, 0, 3, s);
  if (nf && !cheb_coarse) {
    fill<double>(P->Kc, 0.0, nf * nf, s);
    CellArgs<double> a = cell_args<double>(P, c, c.u64, nullptr, nullptr, nullptr);
    P->ops->coarse_assemble(a, P->fmap, nf, P->Kc, (unsigned)c.ncells, s);
    HIPCHECK(hipMemcpyAsync(P->dof_perm, P->dof_of, sizeof(int) * nf, hipMemcpyDeviceToDevice, s));
    const DenseInvWork w{P->gj_P, P->gj_C, P->gj_R, P->sc + SC_TMP, P->gj_sw, P->flag};
    dense_inverse(P->Kc, P->Kinv, nf, P->dof_perm, w, kSingularTol, false, s);
  }
  check_launch("coarse inverse");
}

// Enqueues the copy of what the host half needs into host (setup_host_words doubles).
void setup_copy_back(mfh_problem* P, double* host) {
  const size_t nh = 2 * (size_t)P->d.eig_iters * P->lv.size();
  HIPCHECK(hipMemcpyAsync(host, P->hist, sizeof(double) * nh, hipMemcpyDeviceToHost, P->stream));
  HIPCHECK(hipMemcpyAsync(host + nh, P->flag, 2 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
}

void setup_finish(mfh_problem* P, const double* host) {
  const int nl = (int)P->lv.size();
  const int it = P->d.eig_iters;
  const bool cheb_coarse = P->d.coarse_solver == MFH_COARSE_CHEBYSHEV;
  if (P->eig_fresh) {
    for (int l = 1; l < nl; ++l) {
      Level& v = P->lv[l];
      v.lam_max = lanczos_lambda(host + 2 * (size_t)it * l, it, l);
      set_cheb_coeffs(P, v);
    }
    if (cheb_coarse) {
      Level& c = P->lv[0];
      c.lam_max = lanczos_lambda(host, it, 0, &c.lam_min);
      set_coarse_chebyshev(P, c);
    }
    P->eig_ready = true;
  }
  // caller-fixed estimates replace the Lanczos ones (mfh_set_level_eigenvalues)
  for (int l = 0; l < nl; ++l) {
    Level& v = P->lv[l];
    if (!(v.fix_max > 0)) continue;
    v.lam_max = v.fix_max;
    if (l > 0) {
      set_cheb_coeffs(P, v);
    } else if (cheb_coarse) {
      v.lam_min = v.fix_min;
      set_coarse_chebyshev(P, v);
    }
  }
  int flag[2];
  std::memcpy(flag, host + 2 * (size_t)it * nl, sizeof flag);
  P->coarse_negative = cheb_coarse ? 0 : flag[1];
  if (!cheb_coarse && flag[0]) throw Error(MFH_ERR_NOT_SPD, "coarse-level tangent is numerically singular");
  P->precond_ready = true;
}

void setup_precond(mfh_problem* P) {
  if (P->precond_ready) return;
  setup_enqueue(P);
  std::vector<double> host(setup_host_words(P));
  setup_copy_back(P, host.data());
  HIPCHECK(hipStreamSynchronize(P->stream));
  setup_finish(P, host.data());
}

// z = V-cycle(r) on the CG's own vectors (r = cg_r, z = cg_z); replays the
// captured graph when graphs are enabled and the stream can be captured.
bool graphs_on(const mfh_problem* P) { return P->use_graphs && P->stream != nullptr; }

void capture_vcycle(mfh_problem* P) {
  if (!graphs_on(P) || P->graph_ready) return;
  HIPCHECK(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
  vcycle(P, P->cg_r, P->cg_z);
  HIPCHECK(hipStreamEndCapture(P->stream, &P->graph));
  HIPCHECK(hipGraphInstantiate(&P->gexec, P->graph, nullptr, nullptr, 0));
  P->graph_ready = true;
}

void precond(mfh_problem* P) {
  if (graphs_on(P)) {
    capture_vcycle(P);
    HIPCHECK(hipGraphLaunch(P->gexec, P->stream));
  } else {
    vcycle(P, P->cg_r, P->cg_z);
  }
}

struct CgResult {
  int iters = 0;
  double relres = 0;
  mfh_status st = MFH_OK;
};

// Enqueued pieces of the preconditioned CG (Hestenes-Stiefel, x0 = 0) on the
// problem's own vectors; the single-problem solve and the batched lockstep
// solve issue the same sequence per problem.
void cg_start(mfh_problem* P, const double* b, double* x) {   // x = 0, r = b, bb = b.b
  const long long n = P->lv.back().ndofs;
  fill<double>(x, 0.0, n, P->stream);
  HIPCHECK(hipMemcpyAsync(P->cg_r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, P->stream));
  dot<double, double>(b, b, n, P->part, P->sc + SC_BB, P->stream);
}

void cg_first_dir(mfh_problem* P) {   // z = M r, p = z, rz = r.z
  const long long n = P->lv.back().ndofs;
  precond(P);
  HIPCHECK(hipMemcpyAsync(P->cg_p, P->cg_z, sizeof(double) * n, hipMemcpyDeviceToDevice, P->stream));
  dot<double, double>(P->cg_r, P->cg_z, n, P->part, P->sc + SC_RZ, P->stream);
}

void cg_step(mfh_problem* P, double* x) {   // Ap = K p, alpha = rz / pAp, x += alpha p, r -= alpha Ap, rr
  const long long n = P->lv.back().ndofs;
  vmult<double>(P, (int)P->lv.size() - 1, P->cg_p, P->cg_Ap);
  dot<double, double>(P->cg_p, P->cg_Ap, n, P->part, P->sc + SC_PAP, P->stream);
  scalar_div(P->sc, SC_ALPHA, SC_RZ, SC_PAP, -1, -1, nullptr, 0, P->stream);
  cg_update<double>(x, P->cg_r, P->cg_p, P->cg_Ap, n, P->sc, P->part, P->stream);
}

void cg_next_dir(mfh_problem* P) {   // z = M r, beta = r.z / rz, p = z + beta p
  const long long n = P->lv.back().ndofs;
  precond(P);
  dot<double, double>(P->cg_r, P->cg_z, n, P->part, P->sc + SC_RZNEW, P->stream);
  scalar_div(P->sc, SC_BETA, SC_RZNEW, SC_RZ, SC_RZ, SC_RZNEW, nullptr, 0, P->stream);
  cg_pupdate<double>(P->cg_p, P->cg_z, n, P->sc, P->stream);
}

void cg_true_residual(mfh_problem* P, const double* b, const double* x) {   // |b - K_c x|^2 into SC_TMP
  const long long n = P->lv.back().ndofs;
  vmult<double>(P, (int)P->lv.size() - 1, x, P->cg_Ap);
  lincomb3<double>(P->cg_r, 1.0, b, -1.0, P->cg_Ap, 0.0, nullptr, n, P->stream);
  dot<double, double>(P->cg_r, P->cg_r, n, P->part, P->sc + SC_TMP, P->stream);
}

// Host decision after an iteration: BREAKDOWN, OK (converged), NOT_CONVERGED
// (budget spent) or 1 (continue).
int cg_judge(const double* h, double bb, int it, double rtol, int max_it, double* relres) {
  const double pAp = h[SC_PAP], rr = h[SC_RR];
  if (!(pAp > 0) || !std::isfinite(rr)) return MFH_ERR_BREAKDOWN;
  *relres = std::sqrt(rr / bb);
  if (*relres <= rtol) return MFH_OK;
  if (it == max_it) return MFH_ERR_NOT_CONVERGED;
  return 1;
}

CgResult cg_solve(mfh_problem* P, const double* b, double* x, double rtol, int max_it) {
  hipStream_t s = P->stream;
  CgResult res;
  cg_start(P, b, x);
  const double bb = read_scalar(P, P->sc + SC_BB);
  if (!std::isfinite(bb)) {
    res.st = MFH_ERR_BREAKDOWN;
    res.relres = NAN;
    return res;
  }
  if (bb == 0.0) return res;
  cg_first_dir(P);
  res.st = MFH_ERR_NOT_CONVERGED;
  for (int it = 1; it <= max_it; ++it) {
    cg_step(P, x);
    double h[SC_COUNT];
    HIPCHECK(hipMemcpyAsync(h, P->sc, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    res.iters = it;
    const int j = cg_judge(h, bb, it, rtol, max_it, &res.relres);
    if (j != 1) {
      res.st = (mfh_status)j;
      break;
    }
    cg_next_dir(P);
  }
  cg_true_residual(P, b, x);
  const double rr = read_scalar(P, P->sc + SC_TMP);
  if (res.st != MFH_ERR_BREAKDOWN) res.relres = std::sqrt(rr / bb);
  check_launch("cg");
  return res;
}

double norm2(mfh_problem* P, const double* v, long long n) {
  dot<double, double>(v, v, n, P->part, P->sc + SC_TMP, P->stream);
  return std::sqrt(read_scalar(P, P->sc + SC_TMP));
}

template <typename F>
mfh_status guarded(mfh_problem* P, F&& f) {
  try {
    f();
    if (P) P->err.clear();
    return MFH_OK;
  } catch (const Error& e) {
    if (P)
      P->err = e.what();
    else
      g_err = e.what();
    return e.st;
  } catch (const std::exception& e) {
    if (P)
      P->err = e.what();
    else
      g_err = e.what();
    return MFH_ERR_INVALID_ARG;
  }
}

// Row pointer of the CSR form of K_c on a level (see csr_pattern): a free row
// holds dim * prod over the axes of the node range of the cells holding its
// node, a constrained row its diagonal.
std::vector<long long> csr_row_ptr(const mfh_problem* P, const Level& v) {
  const int p = P->d.degree, L = v.L, dim = P->d.dim;
  std::vector<long long> len(L);
  for (int I = 0; I < L; ++I) {
    const int lo = I % p ? I - I % p : std::max(0, I - p);
    const int hi = I % p ? lo + p : std::min(L - 1, I + p);
    len[I] = hi - lo + 1;
  }
  std::vector<long long> rp(v.ndofs + 1);
  rp[0] = 0;
  long long r = 0;
  for (int c = 0; c < dim; ++c)
    for (int K = 0; K < (dim == 3 ? L : 1); ++K)
      for (int J = 0; J < L; ++J)
        for (int I = 0; I < L; ++I, ++r) {
          unsigned f = (I == 0 ? 1u : 0u) | (I == L - 1 ? 2u : 0u) | (J == 0 ? 4u : 0u) | (J == L - 1 ? 8u : 0u);
          if (dim == 3) f |= (K == 0 ? 16u : 0u) | (K == L - 1 ? 32u : 0u);
          const long long n = (f & v.lt.fmask[c]) ? 1 : dim * len[I] * len[J] * (dim == 3 ? len[K] : 1);
          rp[r + 1] = rp[r] + n;
        }
  return rp;
}

// Lanes per row of the CSR SpMV: 16 for mean rows up to 100 entries, else 8
// (measured on the 3-D lattice patterns of degrees 1 to 4).
int csr_group(const mfh_problem* P) {
  const int p = P->d.degree, dim = P->d.dim;
  const double ml = (double)(2 * p + 1 + (p - 1) * (p + 1)) / p;   // mean node range per axis (interior)
  return dim * std::pow(ml, dim) <= 100.0 ? 16 : 8;
}

void need(bool c, const char* m) {
  if (!c) throw Error(MFH_ERR_INVALID_ARG, m);
}

void check_level(const mfh_problem* P, int level) {
  need(level >= 0 && level < (int)P->lv.size(), "level out of range");
}

}  // namespace
}  // namespace mfh

using namespace mfh;

extern "C" {

void mfh_desc_defaults(mfh_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->n_levels = 1;
  d->n_materials = 1;
  d->qp_policy = MFH_QP_RECOMPUTE;
  d->scatter = MFH_SCATTER_AUTO;
  d->vcycle_dtype = MFH_F32;
  d->cheb_degree = 4;
  d->n_smooth = 2;
  d->eig_iters = 30;
  d->cheb_lo = 0.6;
  d->cheb_hi = 1.2;
  d->level_field = MFH_LEVEL_FIELD_NODAL;
  d->coarse_solver = MFH_COARSE_DIRECT;
  d->eig_refresh = 1;
  d->law = MFH_LAW_NEO_HOOKE;
  d->tile_shape = MFH_TILE_SHAPE_AUTO;
  d->cell_block = MFH_CELL_BLOCK_AUTO;
}

mfh_status mfh_workspace_size(const mfh_desc* desc, size_t* bytes) {
  return guarded(nullptr, [&] {
    validate(desc);
    need(bytes != nullptr, "bytes is NULL");
    mfh_problem tmp;
    tmp.d = *desc;
    build_host(&tmp);
    *bytes = layout(&tmp, nullptr);
  });
}

mfh_status mfh_create(const mfh_desc* desc, void* ws, size_t bytes, void* stream, mfh_problem** out) {
  std::unique_ptr<mfh_problem> P(new mfh_problem());
  mfh_status st = guarded(nullptr, [&] {
    validate(desc);
    need(out != nullptr, "out is NULL");
    need(ws != nullptr, "workspace is NULL");
    need((reinterpret_cast<uintptr_t>(ws) & 255) == 0, "workspace must be 256-byte aligned");
    P->d = *desc;
    P->mu.assign(desc->mu, desc->mu + desc->n_materials);
    P->lam.assign(desc->lambda, desc->lambda + desc->n_materials);
    if (desc->law == MFH_LAW_MOONEY_RIVLIN)
      P->mu2.assign(desc->mu2, desc->mu2 + desc->n_materials);
    else
      P->mu2.assign(desc->n_materials, 0.0);
    P->d.mu = P->d.lambda = P->d.mu2 = P->d.inclusions = nullptr;   // caller's arrays: copied above
    P->incl.assign(desc->inclusions, desc->inclusions + (size_t)desc->n_inclusions * (desc->dim + 2));
    P->stream = static_cast<hipStream_t>(stream);
    build_host(P.get());
    const size_t need_bytes = layout(P.get(), nullptr);
    if (bytes < need_bytes)
      throw Error(MFH_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need_bytes) + " bytes");
    layout(P.get(), static_cast<char*>(ws));
    hipStream_t s = P->stream;
    if (!P->incl.empty())
      HIPCHECK(hipMemcpyAsync(P->incl_dev, P->incl.data(), sizeof(double) * P->incl.size(), hipMemcpyHostToDevice, s));
    for (Level& v : P->lv) {
      material_bits(v.bits, v.ncells, v.N, desc->dim, desc->degree + 1, P->tb64, v.h, P->incl_dev,
                    desc->n_inclusions, v.nwords, s);
      for (DevBand* db : {&v.P1, &v.R1, &v.I1}) {
        if (!db->nout) continue;
        std::vector<float> v32(db->host.vals.begin(), db->host.vals.end());
        HIPCHECK(hipMemcpyAsync(db->start, db->host.start.data(), sizeof(int) * db->nout, hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(db->v64, db->host.vals.data(), sizeof(double) * db->host.vals.size(),
                                hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(db->v32, v32.data(), sizeof(float) * v32.size(), hipMemcpyHostToDevice, s));
        HIPCHECK(hipStreamSynchronize(s));
      }
    }
    const Level& c = P->lv[0];
    if (P->has_coarse)
      HIPCHECK(hipMemcpyAsync(P->fmap, P->h_fmap.data(), sizeof(int) * c.ndofs, hipMemcpyHostToDevice, s));
    if (P->nf)
      HIPCHECK(hipMemcpyAsync(P->dof_of, P->h_dof_of.data(), sizeof(int) * P->nf, hipMemcpyHostToDevice, s));
    check_launch("create");
    HIPCHECK(hipStreamSynchronize(s));
    *out = P.release();
  });
  return st;
}

mfh_status mfh_destroy(mfh_problem* P) {
  delete P;
  return MFH_OK;
}

mfh_status mfh_n_dofs(const mfh_problem* P, int level, long long* n) {
  return guarded(const_cast<mfh_problem*>(P), [&] {
    need(P && n, "NULL argument");
    check_level(P, level);
    *n = P->lv[level].ndofs;
  });
}

mfh_status mfh_set_deformation(mfh_problem* P, const double* u, double* min_J) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(u != nullptr, "u is NULL");
    const double mj = set_deformation(P, u);
    if (min_J) *min_J = mj;
  });
}

mfh_status mfh_tangent_vmult(mfh_problem* P, int level, int dtype, const void* x, void* y) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    check_level(P, level);
    need(x && y, "x/y is NULL");
    need(x != y, "x and y must not overlap");
    need(P->deformed, "set_deformation has not succeeded yet");
    if (dtype == MFH_F64)
      vmult<double>(P, level, static_cast<const double*>(x), static_cast<double*>(y));
    else if (dtype == MFH_F32)
      vmult<float>(P, level, static_cast<const float*>(x), static_cast<float*>(y));
    else
      need(false, "dtype must be MFH_F64 or MFH_F32");
    check_launch("tangent_vmult");
  });
}

mfh_status mfh_csr_size(mfh_problem* P, int level, long long* n_rows, long long* nnz) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    check_level(P, level);
    need(n_rows && nnz, "n_rows/nnz is NULL");
    Level& v = P->lv[level];
    if (v.csr_nnz < 0) v.csr_nnz = csr_row_ptr(P, v).back();   // O(rows) on the host: once per level
    *n_rows = v.ndofs;
    *nnz = v.csr_nnz;
  });
}

mfh_status mfh_csr_assemble(mfh_problem* P, int level, long long* row_ptr, int* col, double* val) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    check_level(P, level);
    need(row_ptr && col && val, "row_ptr/col/val is NULL");
    need(P->deformed, "set_deformation has not succeeded yet");
    const Level& v = P->lv[level];
    need(v.ndofs < (1LL << 31), "more than 2^31 - 1 rows: the column indices are int32");
    const std::vector<long long> rp = csr_row_ptr(P, v);
    HIPCHECK(hipMemcpyAsync(row_ptr, rp.data(), sizeof(long long) * rp.size(), hipMemcpyHostToDevice, P->stream));
    HIPCHECK(hipStreamSynchronize(P->stream));   // rp is pageable and local
    csr_pattern(row_ptr, col, val, v.lt, P->d.degree, v.ndofs, P->stream);
    CellArgs<double> a = cell_args<double>(P, v, v.u64, nullptr, nullptr, nullptr);
    P->ops->csr_assemble(a, row_ptr, val, (unsigned)v.ncells, P->stream);
    check_launch("csr_assemble");
    HIPCHECK(hipStreamSynchronize(P->stream));
  });
}

mfh_status mfh_csr_spmv(mfh_problem* P, int level, const long long* row_ptr, const int* col, const double* val,
                        const double* x, double* y) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    check_level(P, level);
    need(row_ptr && col && val && x && y, "row_ptr/col/val/x/y is NULL");
    need(x != y, "x and y must not overlap");
    csr_spmv(row_ptr, col, val, x, y, P->lv[level].ndofs, csr_group(P), P->stream);
    check_launch("csr_spmv");
  });
}

mfh_status mfh_residual(mfh_problem* P, const double* u, double* r) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(u && r, "u/r is NULL");
    need(u != r, "u and r must not overlap");
    residual(P, u, r);
    check_launch("residual");
  });
}

mfh_status mfh_gmg_vcycle(mfh_problem* P, const double* r, double* z) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(r && z, "r/z is NULL");
    need(r != z, "r and z must not overlap");
    need(P->deformed, "set_deformation has not succeeded yet");
    need(P->has_coarse, "coarsest level too large for the direct solve: use more levels");
    setup_precond(P);
    if (P->use_graphs && P->stream != nullptr) {
      const long long n = P->lv.back().ndofs;
      HIPCHECK(hipMemcpyAsync(P->cg_r, r, sizeof(double) * n, hipMemcpyDeviceToDevice, P->stream));
      precond(P);
      HIPCHECK(hipMemcpyAsync(z, P->cg_z, sizeof(double) * n, hipMemcpyDeviceToDevice, P->stream));
    } else {
      vcycle(P, r, z);
    }
    check_launch("gmg_vcycle");
  });
}

mfh_status mfh_cg_solve(mfh_problem* P, const double* b, double* x, double rtol, int max_it, int* iters,
                        double* relres) {
  if (!P) return MFH_ERR_INVALID_ARG;
  mfh_status st = MFH_OK;
  mfh_status g = guarded(P, [&] {
    need(b && x, "b/x is NULL");
    need(b != x, "b and x must not overlap");
    need(max_it >= 1 && rtol >= 0, "need max_it >= 1 and rtol >= 0");
    need(P->deformed, "set_deformation has not succeeded yet");
    need(P->has_coarse, "coarsest level too large for the direct solve: use more levels");
    setup_precond(P);
    CgResult r = cg_solve(P, b, x, rtol, max_it);
    if (iters) *iters = r.iters;
    if (relres) *relres = r.relres;
    st = r.st;
    if (st == MFH_ERR_NOT_CONVERGED) throw Error(st, "CG did not reach the tolerance within max_it iterations");
    if (st == MFH_ERR_BREAKDOWN) throw Error(st, "CG breakdown (p^T A p <= 0 or NaN)");
  });
  return g;
}

const char* mfh_last_error(const mfh_problem* P) { return P ? P->err.c_str() : g_err.c_str(); }

mfh_status mfh_apply_dirichlet(mfh_problem* P, double* u, const double* fv, double scale) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(u && fv, "NULL argument");
    const Level& v = P->lv.back();
    set_dirichlet(u, v.lt, fv, scale, v.ndofs, P->stream);
    check_launch("apply_dirichlet");
  });
}

// Newton globalisation (the paper does not say how it handles failed steps):
// failed increments are halved down to 1/2^kMaxCut of a load step, and a step length
// alpha = 1, 1/2, ... (at most kMaxHalvings halvings) that keeps J > 0 and,
// once the prescribed values are met, lowers |R|^2 by the Armijo factor
// 1 - 2 kArmijo alpha.
constexpr int kMaxCut = 8;
constexpr int kMaxHalvings = 12;
constexpr double kArmijo = 1e-4;

mfh_status mfh_newton_solve(mfh_problem* P, double* u, const double* fv, const double* ft, int n_steps,
                            double cg_rtol, int cg_max_it, double du_tol, double r_tol, int max_newton,
                            double max_seconds, mfh_newton_record* rec, int max_rec, int* n_rec) {
  if (!P) return MFH_ERR_INVALID_ARG;
  int nrec = 0;
  mfh_status st = guarded(P, [&] {
    need(u && fv, "NULL argument");
    need(n_steps >= 1 && cg_max_it >= 1 && max_newton >= 1, "bad iteration limits");
    need(P->has_coarse, "coarsest level too large for the direct solve: use more levels");
    const Level& v = P->lv.back();
    const long long n = v.ndofs;
    hipStream_t s = P->stream;
    const int top = (int)P->lv.size() - 1;
    const double h0 = 1.0 / n_steps;
    double done = 0.0, h = h0;
    int step = 0, cutbacks = 0;   // increment halvings in the solve
    const auto t_start = Clock::now();
    if (ft) external_force(P, ft, P->f_ext);   // dead tractions scale with the load like fv
    // R(v) = F_int(v) - s f_ext on free rows (constrained rows zero) into Rv
    auto eval_residual = [&](const double* w, double* Rv, double sc) {
      residual(P, w, Rv);
      if (ft) axpby<double>(Rv, P->f_ext, -sc, 1.0, n, s);
    };
    // MFH_NEWTON_LOG=1 in the environment: one line per Newton step on stderr
    const char* log_env = std::getenv("MFH_NEWTON_LOG");
    const bool log = log_env && log_env[0] == '1';
    auto log_step = [&](const mfh_newton_record& r) {
      if (!log) return;
      std::fprintf(stderr,
                   "[mfh newton] load %.6f step %d: |b| %.3e, CG %d (%.1e), alpha %g, |R| %.3e, |du| %.3e, "
                   "min J %.4f, coarse negative %d, %.0f ms\n",
                   r.load_fraction, r.newton_iter, r.residual_norm, r.cg_iters, r.cg_relres, r.step_length,
                   r.residual_after, r.du_norm, r.min_J, r.coarse_negative, r.setup_ms + r.solve_ms + r.residual_ms);
      std::fflush(stderr);
    };
    while (done < 1.0 - 1e-12) {
      const double target = std::fmin(1.0, done + h);
      ++step;
      HIPCHECK(hipMemcpyAsync(P->nw_save, u, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      double R0 = -1;
      bool conv = false;
      bool pending = true;                       // prescribed values of `target` not yet met
      mfh_status fail = MFH_ERR_NOT_CONVERGED;   // why the increment failed
      eval_residual(u, P->nw_R, target);
      double rn = norm2(P, P->nw_R, n);          // |R(u)| on free rows
      for (int it = 0; it < max_newton; ++it) {
        if (max_seconds > 0 && ms_since(t_start) > 1e3 * max_seconds) {
          HIPCHECK(hipMemcpyAsync(u, P->nw_save, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
          HIPCHECK(hipStreamSynchronize(s));
          throw Error(MFH_ERR_NOT_CONVERGED, "time budget exhausted at load fraction " + std::to_string(done));
        }
        mfh_newton_record r{};
        r.load_step = step;
        r.newton_iter = it;
        r.load_fraction = target;
        r.cutbacks = cutbacks;
        r.step_length = NAN;
        auto t0 = Clock::now();
        mfh_status sd = guarded(P, [&] { r.min_J = set_deformation(P, u); });
        if (sd == MFH_ERR_INVERTED) {
          fail = MFH_ERR_INVERTED;
          break;
        }
        if (sd != MFH_OK) throw Error(sd, P->err);
        // a level tangent too indefinite for the eigenvalue estimate (breakdown
        // at its first CG step) or a singular coarse tangent fails the increment
        const mfh_status sp = guarded(P, [&] { setup_precond(P); });
        if (sp == MFH_ERR_BREAKDOWN || sp == MFH_ERR_NOT_SPD) {
          r.residual_norm = r.residual_after = r.cg_relres = NAN;
          r.setup_ms = ms_since(t0);
          if (rec && nrec < max_rec) rec[nrec] = r;
          ++nrec;
          log_step(r);
          fail = sp;
          break;
        }
        if (sp != MFH_OK) throw Error(sp, P->err);
        r.coarse_negative = P->coarse_negative;
        r.setup_ms = ms_since(t0);
        t0 = Clock::now();
        if (pending) {   // carry the rest of the prescribed values linearly: b = -(R + (I - C) K dg)
          dirichlet_delta(u, P->nw_dg, v.lt, fv, target, n, s);
          vmult<double>(P, top, P->nw_dg, P->nw_b, 0);
          lincomb3<double>(P->nw_b, -1.0, P->nw_R, -1.0, P->nw_b, 0.0, nullptr, n, s);
        } else {
          lincomb3<double>(P->nw_b, -1.0, P->nw_R, 0.0, nullptr, 0.0, nullptr, n, s);
        }
        r.residual_norm = norm2(P, P->nw_b, n);
        if (R0 < 0) R0 = r.residual_norm;
        CgResult cr = cg_solve(P, P->nw_b, P->nw_du, cg_rtol, cg_max_it);
        r.cg_iters = cr.iters;
        r.cg_relres = cr.relres;
        r.residual_after = NAN;
        r.solve_ms = ms_since(t0);
        if (cr.st != MFH_OK) {   // breakdown (p^T K p <= 0: the tangent is indefinite here) or no convergence
          if (cr.st == MFH_ERR_BREAKDOWN) r.cg_relres = NAN;
          if (rec && nrec < max_rec) rec[nrec] = r;
          ++nrec;
          log_step(r);
          fail = cr.st;
          break;
        }
        if (pending) axpby<double>(P->nw_du, P->nw_dg, 1.0, 1.0, n, s);   // du = d + dg
        // step length: halve until J > 0 everywhere (finite residual) and, with
        // the prescribed values met, |R|^2 drops by the Armijo factor
        t0 = Clock::now();
        double alpha = 1.0, rt = NAN;
        bool accepted = false;
        for (int k = 0; k <= kMaxHalvings; ++k) {
          lincomb3<double>(P->nw_b, 1.0, u, alpha, P->nw_du, 0.0, nullptr, n, s);   // trial state
          if (alpha == 1.0 && pending) set_dirichlet(P->nw_b, v.lt, fv, target, n, s);
          eval_residual(P->nw_b, P->nw_R, target);
          rt = norm2(P, P->nw_R, n);
          if (std::isfinite(rt) && (pending || rt * rt <= (1.0 - 2.0 * kArmijo * alpha) * rn * rn)) {
            accepted = true;
            break;
          }
          alpha *= 0.5;
        }
        r.residual_ms = ms_since(t0);
        if (!accepted) {   // every trial inverted a quadrature point or failed to lower |R|
          if (rec && nrec < max_rec) rec[nrec] = r;
          ++nrec;
          log_step(r);
          eval_residual(u, P->nw_R, target);   // keep nw_R = R(u) consistent
          fail = std::isfinite(rt) ? MFH_ERR_NOT_CONVERGED : MFH_ERR_INVERTED;
          break;
        }
        HIPCHECK(hipMemcpyAsync(u, P->nw_b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        rn = rt;
        pending = pending && alpha < 1.0;
        r.step_length = alpha;
        r.du_norm = alpha * norm2(P, P->nw_du, n);
        r.residual_after = rt;
        if (rec && nrec < max_rec) rec[nrec] = r;
        ++nrec;
        log_step(r);
        if (!pending && r.du_norm <= du_tol && (rt <= r_tol || rt <= r_tol * R0)) {
          conv = true;
          break;
        }
      }
      if (conv) {
        done = target;
        if (h < h0) h = std::fmin(h0, 2.0 * h);   // grow back after a successful cut increment
        continue;
      }
      // failed: restore the state of the increment's start and halve the increment
      HIPCHECK(hipMemcpyAsync(u, P->nw_save, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
      ++cutbacks;
      if (target - done <= h0 / (1 << kMaxCut) * (1.0 + 1e-9))
        throw Error(fail, std::string("Newton failed: an increment of 1/") + std::to_string(1 << kMaxCut) +
                              " of a load step did not converge at load fraction " + std::to_string(done));
      h = 0.5 * (target - done);
    }
  });
  if (n_rec) *n_rec = nrec;
  return st;
}

mfh_status mfh_external_force(mfh_problem* P, const double* face_traction, double* f) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(face_traction && f, "NULL argument");
    external_force(P, face_traction, P->f_ext);
    HIPCHECK(hipMemcpyAsync(f, P->f_ext, sizeof(double) * P->lv.back().ndofs, hipMemcpyDeviceToDevice, P->stream));
    check_launch("external force");
  });
}

mfh_status mfh_scatter_mode(const mfh_problem* P, int level, int dtype, int* mode) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(const_cast<mfh_problem*>(P), [&] {
    check_level(P, level);
    need(mode != nullptr, "mode is NULL");
    need(dtype == MFH_F64 || dtype == MFH_F32, "dtype must be MFH_F64 or MFH_F32");
    *mode = scatter_mode(P, P->lv[level], dtype == MFH_F64 ? 0 : 1);
  });
}

mfh_status mfh_tile_shape(const mfh_problem* P, int level, int dtype, int* shape, int* cells) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(const_cast<mfh_problem*>(P), [&] {
    check_level(P, level);
    need(shape != nullptr && cells != nullptr, "NULL argument");
    need(dtype == MFH_F64 || dtype == MFH_F32, "dtype must be MFH_F64 or MFH_F32");
    const int t = dtype == MFH_F64 ? 0 : 1;
    *shape = tile_shape(P, P->lv[level], t);
    const TileShape& ts = P->ops->tile_shape[t][*shape];
    cells[0] = ts.tx;
    cells[1] = ts.ty;
    cells[2] = ts.tz;
  });
}

mfh_status mfh_cell_block(const mfh_problem* P, int level, int dtype, int* variant, int* cells) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(const_cast<mfh_problem*>(P), [&] {
    check_level(P, level);
    need(variant != nullptr && cells != nullptr, "NULL argument");
    need(dtype == MFH_F64 || dtype == MFH_F32, "dtype must be MFH_F64 or MFH_F32");
    *variant = cell_block(P, P->lv[level], dtype == MFH_F64 ? 0 : 1);
    *cells = P->ops->cpb[*variant];
  });
}

mfh_status mfh_node_coords_1d(mfh_problem* P, int level, double* x) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    check_level(P, level);
    need(x != nullptr, "x is NULL");
    const std::vector<double> X = lattice_coords(P->lv[level].N, P->d.degree);
    std::memcpy(x, X.data(), sizeof(double) * X.size());
  });
}

mfh_status mfh_level_displacement(mfh_problem* P, int level, double* u) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    check_level(P, level);
    need(u != nullptr, "u is NULL");
    need(P->deformed, "set_deformation has not succeeded yet");
    const Level& v = P->lv[level];
    HIPCHECK(hipMemcpyAsync(u, v.u64, sizeof(double) * v.ndofs, hipMemcpyDeviceToDevice, P->stream));
    HIPCHECK(hipStreamSynchronize(P->stream));
  });
}

mfh_status mfh_level_diagonal(mfh_problem* P, int level, double* dg) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    check_level(P, level);
    need(dg != nullptr, "d is NULL");
    need(P->deformed, "set_deformation has not succeeded yet");
    setup_precond(P);
    const Level& v = P->lv[level];
    HIPCHECK(hipMemcpyAsync(dg, v.diag64, sizeof(double) * v.ndofs, hipMemcpyDeviceToDevice, P->stream));
    HIPCHECK(hipStreamSynchronize(P->stream));
  });
}

mfh_status mfh_level_lambda_max(mfh_problem* P, int level, double* lam) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(level >= 1 && level < (int)P->lv.size(), "level must be 1..n_levels-1");
    need(lam != nullptr, "lam is NULL");
    need(P->deformed, "set_deformation has not succeeded yet");
    setup_precond(P);
    *lam = P->lv[level].lam_max;
  });
}

mfh_status mfh_prolongate(mfh_problem* P, int level, int dtype, const void* x, void* y) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(level >= 1 && level < (int)P->lv.size(), "level must be 1..n_levels-1");
    need(x && y && x != y, "bad x/y");
    if (dtype == MFH_F64)
      prolongate<double>(P, level, static_cast<const double*>(x), static_cast<double*>(y), false);
    else if (dtype == MFH_F32)
      prolongate<float>(P, level, static_cast<const float*>(x), static_cast<float*>(y), false);
    else
      need(false, "bad dtype");
    check_launch("prolongate");
  });
}

mfh_status mfh_restrict(mfh_problem* P, int level, int dtype, const void* x, void* y) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(level >= 1 && level < (int)P->lv.size(), "level must be 1..n_levels-1");
    need(x && y && x != y, "bad x/y");
    if (dtype == MFH_F64)
      restrict_<double>(P, level, static_cast<const double*>(x), static_cast<double*>(y));
    else if (dtype == MFH_F32)
      restrict_<float>(P, level, static_cast<const float*>(x), static_cast<float*>(y));
    else
      need(false, "bad dtype");
    check_launch("restrict");
  });
}

mfh_status mfh_chebyshev(mfh_problem* P, int level, const void* f, void* x) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(level >= 1 && level < (int)P->lv.size(), "level must be 1..n_levels-1");
    need(f && x && f != x, "bad f/x");
    need(P->deformed, "set_deformation has not succeeded yet");
    setup_precond(P);
    if (P->d.vcycle_dtype == MFH_F32)
      cheb_apply<float>(P, level, static_cast<const float*>(f), static_cast<float*>(x), false);
    else
      cheb_apply<double>(P, level, static_cast<const double*>(f), static_cast<double*>(x), false);
    check_launch("chebyshev");
  });
}

mfh_status mfh_set_level_eigenvalues(mfh_problem* P, int level, double lam_min, double lam_max) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(level >= 0 && level < (int)P->lv.size(), "level out of range");
    need(lam_max == 0 || (std::isfinite(lam_max) && lam_max > 0), "lam_max must be 0 (clear) or finite and > 0");
    need(lam_max == 0 || level > 0 || P->d.coarse_solver != MFH_COARSE_CHEBYSHEV ||
             (lam_min > 0 && lam_min < lam_max),
         "the Chebyshev coarse solver needs 0 < lam_min < lam_max");
    Level& v = P->lv[level];
    v.fix_max = lam_max;
    v.fix_min = lam_max == 0 ? 0 : lam_min;
    if (lam_max == 0) P->eig_ready = false;   // back to a fresh Lanczos estimate
    P->precond_ready = false;   // the next solver call rebuilds the smoother coefficients
    P->drop_graph();
  });
}

namespace {
// Layout of the dense-inverse workspace: Pinv, C, R, key, scale (doubles), then
// perm, sw, flag (ints), each slot 256-byte aligned.
size_t dense_inverse_layout(long long n, char* base, mfh::DenseInvWork* w, int** perm) {
  mfh::Bump b;
  b.base = base;
  double* Pinv = b.take<double>(64 * 64);
  double* C = b.take<double>((size_t)n * 64);
  double* R = b.take<double>((size_t)n * 64);
  double* scale = b.take<double>(1);
  int* pm = b.take<int>((size_t)n);
  int* sw = b.take<int>(1 + 4 * 64);
  int* flag = b.take<int>(3);
  if (w) *w = mfh::DenseInvWork{Pinv, C, R, scale, sw, flag};
  if (perm) *perm = pm;
  return b.off + 256;
}

void dense_inverse_run(double* a, double* inv, long long n, char* work, hipStream_t s, int* negative);
}  // namespace

mfh_status mfh_dense_inverse_workspace(long long n, size_t* bytes) {
  return guarded(nullptr, [&] {
    need(bytes != nullptr, "bytes is NULL");
    need(n >= 1 && n <= mfh::kMaxCoarseDofs, "n must be 1..20000");
    *bytes = dense_inverse_layout(n, nullptr, nullptr, nullptr);
  });
}

namespace {
// The dense inverse on work arrays at `work` (layout of dense_inverse_layout);
// every array is written before it is read, the flags by a fill kernel.
void dense_inverse_run(double* a, double* inv, long long n, char* work, hipStream_t s, int* negative) {
  mfh::DenseInvWork w{};
  int* perm = nullptr;
  dense_inverse_layout(n, work, &w, &perm);
  mfh::fill<int>(w.flag, 0, 3, s);
  mfh::iota(perm, n, s);
  mfh::dense_inverse(a, inv, n, perm, w, mfh::kSingularTol, true, s);
  int flag[2];
  HIPCHECK(hipMemcpyAsync(flag, w.flag, sizeof flag, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  *negative = flag[1];
  if (flag[0]) throw Error(MFH_ERR_NOT_SPD, "matrix is numerically singular");
}
}  // namespace

mfh_status mfh_dense_inverse(double* a, double* inv, long long n, void* work, size_t work_bytes, void* stream,
                             int* negative) {
  return guarded(nullptr, [&] {
    need(a && inv && work && negative, "NULL argument");
    need(n >= 1 && n <= mfh::kMaxCoarseDofs, "n must be 1..20000");
    need(a + n * n <= inv || inv + n * n <= a, "a and inv must not overlap");
    need(((uintptr_t)work & 255) == 0, "work must be 256-byte aligned");
    if (work_bytes < dense_inverse_layout(n, nullptr, nullptr, nullptr))
      throw Error(MFH_ERR_WORKSPACE, "work smaller than mfh_dense_inverse_workspace reports");
    dense_inverse_run(a, inv, n, static_cast<char*>(work), static_cast<hipStream_t>(stream), negative);
  });
}

// ---- the same without a workspace (callers that cannot allocate) ----------
// Work arrays for n <= kStaticInvMaxN in one file-scope device array; each GPU
// the library runs on holds its own copy until the process ends.  Host code
// never uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
namespace {
constexpr long long kStaticInvMaxN = 2048;
constexpr size_t kStaticInvBytes = (size_t)9 << 18;   // 2.25 MiB
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) char scratch[kStaticInvBytes];

namespace {
char* scratch_for_current_device() {
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev));
  need(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    need(p != nullptr && ((uintptr_t)p & 255) == 0, "scratch symbol address is not 256-byte aligned");
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

mfh_status mfh_dense_inverse_static(double* a, double* inv, long long n, void* stream, int* negative) {
  return guarded(nullptr, [&] {
    need(a && inv && negative, "NULL argument");
    need(n >= 1 && n <= kStaticInvMaxN, "n must be 1..2048 for the allocation-free dense inverse");
    need(a + n * n <= inv || inv + n * n <= a, "a and inv must not overlap");
    if (dense_inverse_layout(n, nullptr, nullptr, nullptr) > kStaticInvBytes)
      throw Error(MFH_ERR_WORKSPACE, "static scratch smaller than the work arrays");
    dense_inverse_run(a, inv, n, scratch_for_current_device(), static_cast<hipStream_t>(stream), negative);
  });
}

mfh_status mfh_coarse_inertia(mfh_problem* P, int* negative) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(negative != nullptr, "negative is NULL");
    need(P->deformed, "set_deformation has not succeeded yet");
    need(P->d.coarse_solver == MFH_COARSE_DIRECT, "the coarse inertia comes from the direct coarse solve");
    need(P->has_coarse, "coarsest level too large for the direct solve: use more levels");
    setup_precond(P);
    *negative = P->coarse_negative;
  });
}

mfh_status mfh_timer_enable(mfh_problem* P, int enable) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    HIPCHECK(hipStreamSynchronize(P->stream));
    P->ev_used = 0;
    P->timing = enable != 0;
  });
}

mfh_status mfh_timer_read(mfh_problem* P, double* total_ms, long long* launches) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    need(total_ms && launches, "NULL argument");
    HIPCHECK(hipStreamSynchronize(P->stream));
    double t = 0;
    for (size_t i = 0; i + 1 < P->ev_used; i += 2) {
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, P->ev[i], P->ev[i + 1]));
      t += ms;
    }
    *total_ms = t;
    *launches = (long long)(P->ev_used / 2);
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Batches of independent problems.

struct mfh_batch {
  std::vector<mfh_problem*> probs;
  hipStream_t stream = nullptr;
  int policy = 0;
  struct Bin {
    int dim = 0, degree = 0;
    std::vector<int> ids;
    mfh::CellArgs<double>* a64 = nullptr;
    mfh::CellArgs<float>* a32 = nullptr;
    int2* items = nullptr;             // (index in bin, cell block) per workgroup
    void** xs = nullptr;
    void** ys = nullptr;
    long long n_items = 0;
    long long max_cells = 0;           // largest finest-level cell count of the bin's problems
    mfh::GatherItem* g[2] = {nullptr, nullptr};   // node-sum items of the ELEMENT problems, per precision
    long long n_g[2] = {0, 0};
    const mfh::OpFns* ops = nullptr;
    std::vector<const void*> last_x, last_y;   // pointer tables on the device (skip re-upload)
  };
  std::vector<Bin> bins;
  // one persistent launch over all problems (3-D, degrees 1 to 3): argument
  // tables of every problem, (problem, cell block, degree) items by falling
  // degree, pointer tables
  int launch = MFH_BATCH_LAUNCH_AUTO;
  bool fused_ok = false;
  mfh::CellArgs<double>* fa64 = nullptr;
  mfh::CellArgs<float>* fa32 = nullptr;
  int4* fitems = nullptr;
  long long n_fitems = 0;
  void** fxs = nullptr;
  void** fys = nullptr;
  bool foff32[2] = {false, false};
  std::vector<const void*> flast_x, flast_y;
  // output fills of the problems on the atomic scatter, per precision (0 FP64, 1 FP32)
  mfh::FillItem<double>* f64 = nullptr;
  mfh::FillItem<float>* f32 = nullptr;
  long long* foff[2] = {nullptr, nullptr};
  long long fchunks[2] = {0, 0};
  std::vector<int> fill_ids[2];
  std::vector<const void*> last_fx[2], last_fy[2];
  double* pin = nullptr;               // pinned host words, one slot per problem
  std::vector<size_t> slot;            // slot offsets into pin
  std::string err;
  ~mfh_batch() {
    if (pin) (void)hipHostFree(pin);
  }
};

namespace mfh {
namespace {

// The batch follows every problem's own scatter choice for its finest level:
// ELEMENT problems write their element buffers and get a batched node-sum
// pass, the others are scattered with atomics into a pre-filled output.
bool batch_elem(const mfh_problem* P, int t) { return scatter_mode(P, P->lv.back(), t) == MFH_SCATTER_ELEMENT; }

long long gather_blocks(const mfh_problem* P) {
  const long long L = P->lv.back().L;
  return ((L * L + kBlock - 1) / kBlock) * (P->d.dim == 3 ? L : 1);
}

size_t batch_layout(mfh_batch* B, char* base) {
  Bump b;
  b.base = base;
  for (auto& bin : B->bins) {
    const size_t nb = bin.ids.size();
    bin.a64 = b.take<CellArgs<double>>(nb);
    bin.a32 = b.take<CellArgs<float>>(nb);
    bin.n_items = 0;
    bin.max_cells = 0;
    bin.n_g[0] = bin.n_g[1] = 0;
    for (int i : bin.ids) {
      const mfh_problem* P = B->probs[i];
      bin.n_items += (P->lv.back().ncells + P->ops->cpb[0] - 1) / P->ops->cpb[0];
      bin.max_cells = std::max(bin.max_cells, P->lv.back().ncells);
      for (int t = 0; t < 2; ++t)
        if (batch_elem(P, t)) bin.n_g[t] += gather_blocks(P);
    }
    bin.items = b.take<int2>(bin.n_items);
    for (int t = 0; t < 2; ++t) bin.g[t] = b.take<GatherItem>(bin.n_g[t]);
    bin.xs = b.take<void*>(nb);
    bin.ys = b.take<void*>(nb);
  }
  for (int t = 0; t < 2; ++t) {
    B->fill_ids[t].clear();
    for (int i = 0; i < (int)B->probs.size(); ++i)
      if (!batch_elem(B->probs[i], t)) B->fill_ids[t].push_back(i);
    B->foff[t] = b.take<long long>(B->fill_ids[t].size() + 1);
  }
  B->f64 = b.take<FillItem<double>>(B->fill_ids[0].size());
  B->f32 = b.take<FillItem<float>>(B->fill_ids[1].size());
  // the fused persistent launch covers 3-D problems of degrees 1 to 3
  B->fused_ok = true;
  B->n_fitems = 0;
  for (const mfh_problem* P : B->probs) {
    B->fused_ok = B->fused_ok && P->d.dim == 3 && P->d.degree <= 3;
    B->n_fitems += (P->lv.back().ncells + P->ops->cpb[0] - 1) / P->ops->cpb[0];
  }
  const size_t n = B->probs.size();
  B->fa64 = b.take<CellArgs<double>>(n);
  B->fa32 = b.take<CellArgs<float>>(n);
  B->fitems = b.take<int4>(B->fused_ok ? B->n_fitems : 0);
  B->fxs = b.take<void*>(n);
  B->fys = b.take<void*>(n);
  return b.off + 256;
}

// Launch form of the batched vmult: the caller's choice, else the tuned one.
bool batch_fused(const mfh_batch* B) {
  if (!B->fused_ok) return false;
  if (B->launch == MFH_BATCH_LAUNCH_AUTO) return kTunedBatchFused;
  return B->launch == MFH_BATCH_LAUNCH_FUSED;
}

void batch_bins(mfh_batch* B) {
  B->bins.clear();
  for (int i = 0; i < (int)B->probs.size(); ++i) {
    const mfh_problem* P = B->probs[i];
    mfh_batch::Bin* bin = nullptr;
    for (auto& x : B->bins)
      if (x.dim == P->d.dim && x.degree == P->d.degree) bin = &x;
    if (!bin) {
      B->bins.emplace_back();
      bin = &B->bins.back();
      bin->dim = P->d.dim;
      bin->degree = P->d.degree;
      bin->ops = P->ops;
    }
    bin->ids.push_back(i);
  }
}

template <typename T>
void batch_vmult(mfh_batch* B, const void* const* x, void* const* y) {
  hipStream_t s = B->stream;
  const int ti = std::is_same<T, double>::value ? 0 : 1;
  // output fill (0, or x on constrained DoFs) of the atomic-scatter problems;
  // the fill table is uploaded only when the pointers change
  const std::vector<int>& fid = B->fill_ids[ti];
  if (!fid.empty()) {
    std::vector<const void*> fx(fid.size()), fy(fid.size());
    for (size_t k = 0; k < fid.size(); ++k) {
      fx[k] = x[fid[k]];
      fy[k] = y[fid[k]];
    }
    FillItem<T>* fdev = ti == 0 ? reinterpret_cast<FillItem<T>*>(B->f64) : reinterpret_cast<FillItem<T>*>(B->f32);
    if (fx != B->last_fx[ti] || fy != B->last_fy[ti]) {
      std::vector<FillItem<T>> items(fid.size());
      for (size_t k = 0; k < fid.size(); ++k) {
        const Level& v = B->probs[fid[k]]->lv.back();
        items[k] = FillItem<T>{static_cast<T*>(y[fid[k]]), static_cast<const T*>(x[fid[k]]), v.lt, v.ndofs};
      }
      HIPCHECK(hipMemcpyAsync(fdev, items.data(), sizeof(FillItem<T>) * fid.size(), hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));   // the host table goes out of scope
      B->last_fx[ti] = fx;
      B->last_fy[ti] = fy;
    }
    fill_dirichlet_batch<T>(fdev, B->foff[ti], (int)fid.size(), B->fchunks[ti], s);
  }
  const bool fused = batch_fused(B);
  if (fused) {   // one persistent launch for the cell blocks of every problem
    const size_t n = B->probs.size();
    std::vector<const void*> xs(x, x + n), ys(y, y + n);
    if (xs != B->flast_x || ys != B->flast_y) {
      HIPCHECK(hipMemcpyAsync(B->fxs, xs.data(), sizeof(void*) * n, hipMemcpyHostToDevice, s));
      HIPCHECK(hipMemcpyAsync(B->fys, ys.data(), sizeof(void*) * n, hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
      B->flast_x = xs;
      B->flast_y = ys;
    }
    const CellArgs<T>* fa = ti == 0 ? reinterpret_cast<const CellArgs<T>*>(B->fa64)
                                    : reinterpret_cast<const CellArgs<T>*>(B->fa32);
    tangent_batch_fused<T>(B->policy, B->foff32[ti], fa, B->fitems, (int)B->n_fitems,
                           reinterpret_cast<const T* const*>(B->fxs), reinterpret_cast<T* const*>(B->fys), s);
  }
  for (auto& bin : B->bins) {
    const size_t nb = bin.ids.size();
    std::vector<const void*> xs(nb), ys(nb);
    for (size_t k = 0; k < nb; ++k) {
      xs[k] = x[bin.ids[k]];
      ys[k] = y[bin.ids[k]];
    }
    if (xs != bin.last_x || ys != bin.last_y) {
      HIPCHECK(hipMemcpyAsync(bin.xs, xs.data(), sizeof(void*) * nb, hipMemcpyHostToDevice, s));
      HIPCHECK(hipMemcpyAsync(bin.ys, ys.data(), sizeof(void*) * nb, hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
      bin.last_x = xs;
      bin.last_y = ys;
    }
    if (fused) {   // only the node sums of the ELEMENT problems remain per bin
      if (ti == 0 && bin.n_g[0])
        bin.ops->elem_gather_batch_d(bin.a64, bin.g[0], reinterpret_cast<const double* const*>(bin.xs),
                                     reinterpret_cast<double* const*>(bin.ys), (unsigned)bin.n_g[0], s);
      if (ti == 1 && bin.n_g[1])
        bin.ops->elem_gather_batch_f(bin.a32, bin.g[1], reinterpret_cast<const float* const*>(bin.xs),
                                     reinterpret_cast<float* const*>(bin.ys), (unsigned)bin.n_g[1], s);
      continue;
    }
    if (ti == 0) {
      bin.ops->tangent_batch_d[B->policy](bin.a64, bin.items, reinterpret_cast<const double* const*>(bin.xs),
                                          reinterpret_cast<double* const*>(bin.ys), (unsigned)bin.n_items,
                                          bin.max_cells, s);
      if (bin.n_g[0])
        bin.ops->elem_gather_batch_d(bin.a64, bin.g[0], reinterpret_cast<const double* const*>(bin.xs),
                                     reinterpret_cast<double* const*>(bin.ys), (unsigned)bin.n_g[0], s);
    } else {
      bin.ops->tangent_batch_f[B->policy](bin.a32, bin.items, reinterpret_cast<const float* const*>(bin.xs),
                                          reinterpret_cast<float* const*>(bin.ys), (unsigned)bin.n_items,
                                          bin.max_cells, s);
      if (bin.n_g[1])
        bin.ops->elem_gather_batch_f(bin.a32, bin.g[1], reinterpret_cast<const float* const*>(bin.xs),
                                     reinterpret_cast<float* const*>(bin.ys), (unsigned)bin.n_g[1], s);
    }
  }
  check_launch("batch tangent_vmult");
}

template <typename F>
mfh_status batch_guarded(mfh_batch* B, F&& f) {
  try {
    f();
    if (B) B->err.clear();
    return MFH_OK;
  } catch (const Error& e) {
    if (B) B->err = e.what(); else g_err = e.what();
    return e.st;
  } catch (const std::exception& e) {
    if (B) B->err = e.what(); else g_err = e.what();
    return MFH_ERR_INVALID_ARG;
  }
}

void batch_validate(int n, mfh_problem* const* probs) {
  need(n >= 1 && probs != nullptr, "need n >= 1 problems");
  for (int i = 0; i < n; ++i) {
    need(probs[i] != nullptr, "NULL problem in batch");
    need(probs[i]->d.qp_policy == probs[0]->d.qp_policy, "all problems of a batch must use one qp_policy");
  }
}

// Waits for every listed problem's stream.
void sync_all(mfh_batch* B, const std::vector<int>& ids) {
  for (int i : ids) HIPCHECK(hipStreamSynchronize(B->probs[i]->stream));
}

// Per-problem statuses -> the batch status: the first failing problem's.
void batch_raise(mfh_batch* B, const std::vector<mfh_status>& st, const std::vector<std::string>& msg) {
  for (size_t i = 0; i < st.size(); ++i)
    if (st[i] != MFH_OK) throw Error(st[i], "problem " + std::to_string(i) + ": " + msg[i]);
}

}  // namespace
}  // namespace mfh

extern "C" {

mfh_status mfh_enable_graphs(mfh_problem* P, int enable) {
  if (!P) return MFH_ERR_INVALID_ARG;
  return guarded(P, [&] {
    P->drop_graph();
    P->use_graphs = enable != 0;
  });
}

mfh_status mfh_batch_workspace_size(int n, mfh_problem* const* probs, size_t* bytes) {
  return batch_guarded(nullptr, [&] {
    batch_validate(n, probs);
    need(bytes != nullptr, "bytes is NULL");
    mfh_batch tmp;
    tmp.probs.assign(probs, probs + n);
    batch_bins(&tmp);
    *bytes = batch_layout(&tmp, nullptr);
  });
}

mfh_status mfh_batch_create(int n, mfh_problem* const* probs, void* ws, size_t bytes, void* stream,
                            mfh_batch** out) {
  std::unique_ptr<mfh_batch> B(new mfh_batch());
  mfh_status st = batch_guarded(nullptr, [&] {
    batch_validate(n, probs);
    need(out != nullptr && ws != nullptr, "NULL argument");
    need((reinterpret_cast<uintptr_t>(ws) & 255) == 0, "workspace must be 256-byte aligned");
    B->probs.assign(probs, probs + n);
    B->stream = static_cast<hipStream_t>(stream);
    B->policy = probs[0]->d.qp_policy;
    batch_bins(B.get());
    const size_t need_bytes = batch_layout(B.get(), nullptr);
    if (bytes < need_bytes) throw Error(MFH_ERR_WORKSPACE, "batch workspace too small: need " + std::to_string(need_bytes));
    batch_layout(B.get(), static_cast<char*>(ws));
    hipStream_t s = B->stream;
    for (auto& bin : B->bins) {
      const size_t nb = bin.ids.size();
      need(bin.n_items < (1ll << 31), "batch bin has too many cell blocks");
      std::vector<CellArgs<double>> a64(nb);
      std::vector<CellArgs<float>> a32(nb);
      need(bin.n_g[0] < (1ll << 31) && bin.n_g[1] < (1ll << 31), "batch bin has too many node blocks");
      std::vector<int2> items;
      items.reserve(bin.n_items);
      std::vector<GatherItem> g[2];
      for (size_t k = 0; k < nb; ++k) {
        const mfh_problem* P = B->probs[bin.ids[k]];
        const Level& v = P->lv.back();
        a64[k] = cell_args<double>(P, v, v.u64, v.cache64, nullptr, nullptr);
        a32[k] = cell_args<float>(P, v, v.u32, v.cache32, nullptr, nullptr);
        if (batch_elem(P, 0)) a64[k].elem = P->elem;
        if (batch_elem(P, 1)) a32[k].elem = reinterpret_cast<float*>(P->elem);
        const long long nblk = (v.ncells + P->ops->cpb[0] - 1) / P->ops->cpb[0];
        for (long long j = 0; j < nblk; ++j) items.push_back(make_int2((int)k, (int)j));
        const unsigned L = (unsigned)v.L;
        const unsigned magic = (unsigned)((((unsigned long long)1 << 32) + L - 1) / L);
        const int pblocks = (int)((L * L + kBlock - 1) / kBlock);
        for (int t = 0; t < 2; ++t) {
          if (!batch_elem(P, t)) continue;
          for (int kk = 0; kk < (P->d.dim == 3 ? (int)L : 1); ++kk)
            for (int blk = 0; blk < pblocks; ++blk) g[t].push_back(GatherItem{(int)k, kk, blk, magic});
        }
      }
      HIPCHECK(hipMemcpyAsync(bin.a64, a64.data(), sizeof(CellArgs<double>) * nb, hipMemcpyHostToDevice, s));
      HIPCHECK(hipMemcpyAsync(bin.a32, a32.data(), sizeof(CellArgs<float>) * nb, hipMemcpyHostToDevice, s));
      HIPCHECK(hipMemcpyAsync(bin.items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, s));
      for (int t = 0; t < 2; ++t)
        if (!g[t].empty())
          HIPCHECK(hipMemcpyAsync(bin.g[t], g[t].data(), sizeof(GatherItem) * g[t].size(), hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));   // the host tables above go out of scope
    }
    {   // tables of the fused persistent launch
      const size_t np = B->probs.size();
      std::vector<CellArgs<double>> a64(np);
      std::vector<CellArgs<float>> a32(np);
      std::vector<int4> items;
      B->foff32[0] = B->foff32[1] = true;
      for (size_t i = 0; i < np; ++i) {
        const mfh_problem* P = B->probs[i];
        const Level& v = P->lv.back();
        a64[i] = cell_args<double>(P, v, v.u64, v.cache64, nullptr, nullptr);
        a32[i] = cell_args<float>(P, v, v.u32, v.cache32, nullptr, nullptr);
        if (batch_elem(P, 0)) a64[i].elem = P->elem;
        if (batch_elem(P, 1)) a32[i].elem = reinterpret_cast<float*>(P->elem);
        const long long nv = (long long)std::pow(P->d.degree + 1, P->d.dim);
        B->foff32[0] = B->foff32[0] && nv * v.ncells * 2 * (long long)sizeof(double) < (1LL << 32);
        B->foff32[1] = B->foff32[1] && nv * v.ncells * 2 * (long long)sizeof(float) < (1LL << 32);
      }
      if (B->fused_ok) {
        need(B->n_fitems < (1ll << 31), "batch has too many cell blocks");
        items.reserve(B->n_fitems);
        for (int deg = 3; deg >= 1; --deg)   // heaviest items first
          for (size_t i = 0; i < np; ++i) {
            const mfh_problem* P = B->probs[i];
            if (P->d.degree != deg) continue;
            const long long nblk = (P->lv.back().ncells + P->ops->cpb[0] - 1) / P->ops->cpb[0];
            for (long long j = 0; j < nblk; ++j) items.push_back(make_int4((int)i, (int)j, deg, 0));
          }
        HIPCHECK(hipMemcpyAsync(B->fitems, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, s));
      }
      HIPCHECK(hipMemcpyAsync(B->fa64, a64.data(), sizeof(CellArgs<double>) * np, hipMemcpyHostToDevice, s));
      HIPCHECK(hipMemcpyAsync(B->fa32, a32.data(), sizeof(CellArgs<float>) * np, hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));   // the host tables go out of scope
    }
    for (int t = 0; t < 2; ++t) {
      const std::vector<int>& fid = B->fill_ids[t];
      std::vector<long long> foff(fid.size() + 1, 0);
      for (size_t k = 0; k < fid.size(); ++k) {
        const long long nd = B->probs[fid[k]]->lv.back().ndofs;
        foff[k + 1] = foff[k] + (nd + kFillChunk - 1) / kFillChunk;
      }
      B->fchunks[t] = foff.back();
      HIPCHECK(hipMemcpyAsync(B->foff[t], foff.data(), sizeof(long long) * foff.size(), hipMemcpyHostToDevice, s));
      HIPCHECK(hipStreamSynchronize(s));
    }
    // pinned host slots: device scalars, per-level min J, set-up histories
    B->slot.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      const mfh_problem* P = B->probs[i];
      const size_t w = std::max<size_t>({(size_t)SC_COUNT, P->lv.size(), setup_host_words(P)});
      B->slot[i + 1] = B->slot[i] + ((w + 7) & ~size_t(7));
    }
    HIPCHECK(hipHostMalloc((void**)&B->pin, sizeof(double) * B->slot[n], hipHostMallocDefault));
    *out = B.release();
  });
  return st;
}

mfh_status mfh_batch_destroy(mfh_batch* B) {
  delete B;
  return MFH_OK;
}

const char* mfh_batch_last_error(const mfh_batch* B) { return B ? B->err.c_str() : g_err.c_str(); }

mfh_status mfh_batch_set_deformation(mfh_batch* B, const double* const* u, double* min_J) {
  if (!B) return MFH_ERR_INVALID_ARG;
  return batch_guarded(B, [&] {
    need(u != nullptr, "u is NULL");
    const int n = (int)B->probs.size();
    for (int i = 0; i < n; ++i) need(u[i] != nullptr, "u[i] is NULL");
    std::vector<int> all(n);
    for (int i = 0; i < n; ++i) all[i] = i;
    // enqueue every problem's level data, then drain once
    for (int i = 0; i < n; ++i) {
      mfh_problem* P = B->probs[i];
      setdef_enqueue(P, u[i]);
      HIPCHECK(hipMemcpyAsync(B->pin + B->slot[i], P->minj, sizeof(double) * P->lv.size(), hipMemcpyDeviceToHost,
                              P->stream));
    }
    sync_all(B, all);
    std::vector<mfh_status> st(n, MFH_OK);
    std::vector<std::string> msg(n);
    for (int i = 0; i < n; ++i) {
      mfh_problem* P = B->probs[i];
      double mj = 0;
      st[i] = guarded(P, [&] { mj = setdef_finish(P, B->pin + B->slot[i]); });
      msg[i] = P->err;
      if (min_J) min_J[i] = st[i] == MFH_OK ? mj : NAN;
    }
    batch_raise(B, st, msg);
  });
}

mfh_status mfh_contraction_stage(int degree, int mfma, int sweeps, int blocks, float* out, void* stream) {
  return guarded(nullptr, [&] {
    need(degree == 3 || degree == 4, "degree must be 3 or 4");
    need(mfma == 0 || mfma == 1, "mfma must be 0 or 1");
    need(sweeps >= 1 && blocks >= 1, "need sweeps >= 1 and blocks >= 1");
    need(out != nullptr, "out is NULL");
    contraction_stage(degree, mfma, sweeps, blocks, out, static_cast<hipStream_t>(stream));
    check_launch("contraction stage");
  });
}

mfh_status mfh_batch_set_launch(mfh_batch* B, int mode) {
  if (!B) return MFH_ERR_INVALID_ARG;
  return batch_guarded(B, [&] {
    need(mode == MFH_BATCH_LAUNCH_AUTO || mode == MFH_BATCH_LAUNCH_PER_DEGREE || mode == MFH_BATCH_LAUNCH_FUSED,
         "mode must be MFH_BATCH_LAUNCH_AUTO, _PER_DEGREE or _FUSED");
    need(mode != MFH_BATCH_LAUNCH_FUSED || B->fused_ok,
         "the fused launch covers 3-D problems of degrees 1 to 3 only");
    B->launch = mode;
  });
}

mfh_status mfh_batch_tangent_vmult(mfh_batch* B, int dtype, const void* const* x, void* const* y) {
  if (!B) return MFH_ERR_INVALID_ARG;
  return batch_guarded(B, [&] {
    need(x && y, "x/y is NULL");
    for (size_t i = 0; i < B->probs.size(); ++i) {
      need(x[i] && y[i] && x[i] != y[i], "bad x/y pointer");
      need(B->probs[i]->deformed, "set_deformation has not succeeded on every problem");
    }
    if (dtype == MFH_F64)
      batch_vmult<double>(B, x, y);
    else if (dtype == MFH_F32)
      batch_vmult<float>(B, x, y);
    else
      need(false, "dtype must be MFH_F64 or MFH_F32");
  });
}

mfh_status mfh_batch_cg_solve(mfh_batch* B, const double* const* b, double* const* x, double rtol, int max_it,
                              int* iters, double* relres, double* solve_ms) {
  if (!B) return MFH_ERR_INVALID_ARG;
  return batch_guarded(B, [&] {
    need(b && x, "b/x is NULL");
    need(max_it >= 1 && rtol >= 0, "need max_it >= 1 and rtol >= 0");
    const int n = (int)B->probs.size();
    for (int i = 0; i < n; ++i) {
      const mfh_problem* P = B->probs[i];
      need(b[i] && x[i] && b[i] != x[i], "bad b/x pointer");
      need(P->deformed, "set_deformation has not succeeded on every problem");
      need(P->has_coarse, "a coarsest level is too large for the direct solve");
    }
    const auto t0 = Clock::now();
    std::vector<mfh_status> st(n, MFH_OK);
    std::vector<std::string> msg(n);
    std::vector<int> it(n, 0);
    std::vector<double> bb(n, 0.0), rel(n, 0.0), ms(n, 0.0);
    // 1. preconditioner set-up of every problem that needs one: enqueue all, drain once
    std::vector<int> pending;
    for (int i = 0; i < n; ++i) {
      mfh_problem* P = B->probs[i];
      if (P->precond_ready) continue;
      setup_enqueue(P);
      setup_copy_back(P, B->pin + B->slot[i]);
      pending.push_back(i);
    }
    sync_all(B, pending);
    std::vector<int> active;
    for (int i = 0; i < n; ++i) {
      mfh_problem* P = B->probs[i];
      if (!P->precond_ready) st[i] = guarded(P, [&] { setup_finish(P, B->pin + B->slot[i]); });
      if (st[i] == MFH_OK) st[i] = guarded(P, [&] { capture_vcycle(P); });   // streams are idle here
      if (st[i] == MFH_OK)
        active.push_back(i);
      else
        msg[i] = P->err;
    }
    // 2. lockstep PCG: every round issues one iteration of every active
    //    problem on its own stream, then the host judges all of them at once
    for (int i : active) {
      mfh_problem* P = B->probs[i];
      cg_start(P, b[i], x[i]);
      cg_first_dir(P);
      cg_step(P, x[i]);
      HIPCHECK(hipMemcpyAsync(B->pin + B->slot[i], P->sc, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost,
                              P->stream));
    }
    std::vector<int> finishing;   // problems whose explicit final residual is pending
    bool first = true;
    while (!active.empty()) {
      sync_all(B, active);
      const double now = ms_since(t0);
      std::vector<int> still;
      for (int i : active) {
        mfh_problem* P = B->probs[i];
        const double* h = B->pin + B->slot[i];
        if (first) {
          bb[i] = h[SC_BB];
          if (!std::isfinite(bb[i]) || bb[i] == 0.0) {   // as the single solve: no iteration
            if (bb[i] == 0.0) {
              fill<double>(x[i], 0.0, P->lv.back().ndofs, P->stream);
            } else {
              st[i] = MFH_ERR_BREAKDOWN;
              rel[i] = NAN;
              msg[i] = "right-hand side is not finite";
            }
            ms[i] = now;
            continue;
          }
        }
        it[i] += 1;
        const int j = cg_judge(h, bb[i], it[i], rtol, max_it, &rel[i]);
        if (j == 1) {
          cg_next_dir(P);
          cg_step(P, x[i]);
          HIPCHECK(hipMemcpyAsync(B->pin + B->slot[i], P->sc, sizeof(double) * SC_COUNT, hipMemcpyDeviceToHost,
                                  P->stream));
          still.push_back(i);
          continue;
        }
        ms[i] = now;
        st[i] = (mfh_status)j;
        if (j == MFH_ERR_BREAKDOWN) {
          msg[i] = "CG breakdown (p^T A p <= 0 or NaN)";
          continue;
        }
        if (j == MFH_ERR_NOT_CONVERGED) msg[i] = "CG did not reach the tolerance within max_it iterations";
        cg_true_residual(P, b[i], x[i]);
        HIPCHECK(hipMemcpyAsync(B->pin + B->slot[i] + SC_TMP, P->sc + SC_TMP, sizeof(double), hipMemcpyDeviceToHost,
                                P->stream));
        finishing.push_back(i);
      }
      active.swap(still);
      first = false;
    }
    sync_all(B, finishing);
    for (int i : finishing) rel[i] = std::sqrt(B->pin[B->slot[i] + SC_TMP] / bb[i]);
    check_launch("batch cg");
    for (int i = 0; i < n; ++i) {
      if (iters) iters[i] = it[i];
      if (relres) relres[i] = rel[i];
      if (solve_ms) solve_ms[i] = ms[i];
    }
    batch_raise(B, st, msg);
  });
}

}  // extern "C"
