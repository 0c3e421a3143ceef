// Host plan and C ABI of the SBP-SAT FDTD step (see include/sbpfdtd.h).
//
// The plan turns blocks, faces, interfaces, sources and probes into device
// descriptors: per-block closure-row tables (Appendix rows with the Section
// III SAT row changes), a flat tile list over all blocks (one launch per half
// step covers every block), face buffers and gather jobs for interfaces, and
// ring buffers for the per-step energy and probe samples.  Each step enqueues
// [gather E] -> H update -> [gather H] -> E update on the context's stream.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sbpfdtd.h"
#include "plan.h"

namespace sbp {
template <typename T> hipError_t launch_h(const KArgs&, int, int, int, hipStream_t);
template <typename T> hipError_t launch_e(const KArgs&, int, int, int, hipStream_t);
hipError_t launch_finish(const KArgs&, int, int, hipStream_t);
template <typename T>
hipError_t lts_phase(int, int, int, void*, void*, void*, const void*, const void*, void*, void*, double, double,
                     const Tile*, int, const DevBlock*, const LtsBox*, int, int, hipStream_t);
template <typename T>
hipError_t lts_whole(int, int, const void*, void*, const void*, double, const DevBlock*, hipStream_t);
template <typename T>
hipError_t lts_energy(const void*, const void*, const void*, double, const Tile*, int, const DevBlock*, const void*,
                      double, int, int, double*, hipStream_t);
hipError_t lts_store(const double*, int, double*, hipStream_t);
template <typename T> hipError_t launch_fused(const KArgs&, int, int, hipStream_t);
hipError_t launch_sources(const KArgs&, hipStream_t);
template <typename T>
hipError_t launch_adj_objective(const void*, const DevBlock*, int, const int*, double, double*, hipStream_t);
template <typename T>
hipError_t launch_adj_source(void*, const void*, const DevBlock*, const void*, int, const int*, double, hipStream_t);
template <typename T>
hipError_t launch_adj_grad(const void*, const void*, const void*, long long, double*, hipStream_t);
template <typename T>
hipError_t launch_adj_cells(const DevBlock*, const void*, int, double*, double*, hipStream_t);
template <typename T>
hipError_t launch_gather(const DevBlock*, const FaceJob*, const GatherWG*, int, const Taps*, const KArgs&, int,
                         double*, hipStream_t);
}  // namespace sbp

using namespace sbp;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4e-7 * kPi;
constexpr double kC0 = 299792458.0;
const double kEps0 = 1.0 / (kMu0 * kC0 * kC0);

// Kernel kinds of a block (bit 0 per-cell permittivity, 1 general terms,
// 2 interfaces, 3 absorbing layers, 4 TF/SF box, 5 tabled permittivity: set
// by the tile lists for the launch shapes where it pays).
constexpr int kKinds = 64;

// Kinds in tile-list and launch order: the tabled plain kind (33) right
// after the plain kind that reads the permittivity cells (1), so that
// turning the tables on or off leaves the order of the tiles, of the
// launches and so of the energy partial sums unchanged.
struct KindOrder {
  int k[kKinds];
  KindOrder() {
    int n = 0;
    for (int v = 0; v < kKinds; ++v) {
      if (v == 33) continue;
      k[n++] = v;
      if (v == 1) k[n++] = 33;
    }
  }
};
const KindOrder kKindOrder;

struct HostBlock {
  int n[3];
  double h[3], x0[3];
  std::vector<double> eps, mu, sig;
  int faces[6];
  int iface[6];  // index into ifaces or -1
  // complex fields (periodic faces with a Bloch phase): the block holding
  // the other part, and whether this block holds the imaginary part
  int part_of = -1, imag = 0;
  int tfsf = 0;  // holds the total-field / scattered-field box
  // the per-cell permittivity takes at most kCellTab values (in the field
  // precision): byte indices and a table are uploaded beside the cells
  bool tabled = false;
};

// A coupled pair of faces.  Interfaces join two blocks; a periodic axis
// joins a block's two faces of that axis (a == b, fa the high face), and for
// complex fields `partner` is the block holding the other part (im: this
// block holds the imaginary part) with the Bloch phase alpha.
struct HostIface {
  int a, fa, b, fb, ratio;
  int partner = -1, im = 0;
  double alpha = 0.0;
};

struct HostSource {
  int block;
  Source s;
};
struct HostProbe {
  int block;
  Probe p;
};

}  // namespace

struct sbp_ctx {
  sbp_prec prec = SBP_FP64;
  hipStream_t stream = nullptr;
  sbp_alloc_fn alloc = nullptr;
  sbp_free_fn free_fn = nullptr;
  void* user = nullptr;
  int device = 0;
  std::vector<HostBlock> blocks;
  std::vector<HostIface> ifaces;
  std::vector<HostSource> srcs;
  std::vector<HostProbe> prbs;
  bool finalized = false;
  double dt = 0.0;
  long long nstep = 0;
  long history = 0;
  // device buffers
  // field pools: with the one-pass step, step n reads pool (n even) or pool2
  // (n odd) and writes the other; the two-pass step updates in place
  // (pool2 == pool), which keeps mid-size states within the last-level cache
  void* pool = nullptr;
  void* pool2 = nullptr;
  size_t pool_elems = 0;
  void* mat[3] = {nullptr, nullptr, nullptr};
  unsigned char* d_midx = nullptr;  // byte index per cell (tabled blocks)
  void* d_mtab = nullptr;           // kCellTab values per block
  size_t mtab_blocks = 0;
  bool tables_off = false;  // sbp_set_cell_tables(ctx, 0)
  size_t ncells = 0;
  DevBlock* d_blocks = nullptr;
  std::vector<DevBlock> hblocks;
  Tile* d_tiles = nullptr;
  Tile* d_tiles_bare = nullptr;  // same tiles, flags cleared
  std::vector<Tile> bare;
  std::vector<FTile> fbare;
  size_t bare_cap = 0;
  int ntiles = 0;
  int kind_t0[kKinds] = {}, kind_t1[kKinds] = {};  // tile ranges per block kind
  // one-pass step of the plain kinds (0, 1): tile list, ranges per kind
  int fused = 0, fz = 8;  // two passes by default: measured faster on the 256^3 workload
  // local time stepping (sbp_lts_start / sbp_lts_step): the scratch state on
  // which L is applied (with its own face buffers, step counter and one-slot
  // energy ring), w = L (I - P) E^n, two substep vectors, E^{n-1} (the last
  // three on the near boxes only), two E copies for the energy, per-block
  // unit-time-step and coarse-time-step descriptors and near boxes, the
  // tiles that meet the wider boxes (ranges per kind; rebuilt when the tile
  // list changes) and energy partials
  bool lts = false;
  int lts_p = 1;
  double lts_dt = 0.0;
  long lts_every = 0;
  void *lts_s = nullptr, *lts_w = nullptr, *lts_qa = nullptr, *lts_qb = nullptr, *lts_ep = nullptr;
  void* lts_x[2] = {nullptr, nullptr};
  double* lts_face = nullptr;
  StepState* lts_st = nullptr;
  double* lts_ring = nullptr;
  double* lts_part = nullptr;
  DevBlock* lts_blocks = nullptr;   // unit time step (L u)
  DevBlock* lts_cblocks = nullptr;  // the coarse time step (the ordinary step)
  LtsBox* lts_boxes = nullptr;
  std::vector<LtsBox> lts_hbox;  // near boxes (the recursion's nodes)
  std::vector<LtsBox> lts_tbox;  // wider boxes (the operator's tiles)
  Tile* d_near = nullptr;  // tiles meeting the wider boxes (the operator and the phases)
  Tile* d_far = nullptr;   // tiles of the blocks that are not refined (the ordinary step)
  size_t near_cap = 0, far_cap = 0;
  int nnear = 0, nfar = 0;
  int nk_t0[kKinds] = {}, nk_t1[kKinds] = {}, fk_t0x[kKinds] = {}, fk_t1x[kKinds] = {};
  GatherWG* d_nwg[2] = {nullptr, nullptr};  // gather workgroups whose face nodes meet a wider box (E, H)
  GatherWG* d_fwg[2] = {nullptr, nullptr};  // gather workgroups of faces between blocks that are not refined
  int nnwg[2] = {0, 0}, nfwg[2] = {0, 0};
  bool near_dirty = true, near_built = false;
  FTile* d_ftiles = nullptr;
  FTile* d_ftiles_bare = nullptr;
  size_t ftiles_cap = 0;
  int fk_t0[2] = {0, 0}, fk_t1[2] = {0, 0};
  size_t tiles_cap = 0;
  Source* d_src = nullptr;
  double* d_srcval = nullptr;
  int nsrc_total = 0;
  Probe* d_prb = nullptr;
  std::vector<int> probe_order;  // user probe id -> device probe index
  double* d_energy = nullptr;
  double* d_probes = nullptr;
  double* d_partials = nullptr;
  size_t partials_cap = 0;
  size_t partials_need = 0;    // partial sums one step of the current launch shape writes
  double* scratch = nullptr;   // this device's fixed scratch array (sbp_step_static)
  StepState* d_st = nullptr;
  double* d_face = nullptr;
  // convolutional PML (faces set to SBP_CPML): layer parameters, per-block
  // profile tables and recursion variables, both in the field type
  int pml_cells = 10, pml_m = 3;
  double pml_sigma_factor = 0.8, pml_kappa_max = 1.0, pml_alpha_max = 0.0;
  void* d_pml = nullptr;
  void* d_psi = nullptr;
  size_t psi_elems = 0;
  size_t face_elems = 1;
  FaceJob* d_jobs_e = nullptr;
  FaceJob* d_jobs_h = nullptr;
  int njobs_e = 0, njobs_h = 0;
  GatherWG* d_wg_e = nullptr;  // per-workgroup job tables of the two gathers
  GatherWG* d_wg_h = nullptr;
  int nwg_e = 0, nwg_h = 0;
  std::vector<FaceJob> hjobs[2];  // host copies (E, H)
  std::vector<GatherWG> hwg[2];
  Taps* d_taps = nullptr;
  // total-field / scattered-field injection (sbp_set_tfsf): the block, cell
  // box, propagation axis, E polarisation, line margin, the incident source
  // (its cell on the line) and the device line (E then H, fp64)
  bool tf_on = false;
  int tf_block = -1, tf_box[6] = {0, 0, 0, 0, 0, 0}, tf_axis = 0, tf_pol = 0, tf_margin = 16, tf_cell = 0;
  Source tf_srcdef{};
  int tf_sidx = 0, tf_len = 0;
  double* d_line = nullptr;
  TfDesc* d_tf = nullptr;
  int tx = 128, ty = 1, cz = 8, wgs = 0;  // launch shape (sbp_set_launch); fastest measured on 256^3 fp32
  bool launch_set = false;                  // set by sbp_set_launch / sbp_autotune
  std::string err;
  int graph_steps = 0;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  bool profile = false;
  std::vector<hipEvent_t> kev;
  int kev_used = 0;
  std::vector<void*> allocs;
};

namespace {

sbp_status fail(sbp_ctx* c, sbp_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

#define HIPCHK(ctx, expr)                                                               \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(ctx, SBP_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

void* dalloc(sbp_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 8;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (c->alloc) {
    p = c->alloc(bytes, c->user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) c->allocs.push_back(p);
  return p;
}

void dfree(sbp_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  if (c->free_fn) c->free_fn(p, c->user);
  else (void)hipFree(p);
}

size_t elem_size(const sbp_ctx* c) { return c->prec == SBP_FP64 ? 8 : 4; }
// Bytes of the TF/SF incident line (E then H, fp64).
size_t line_bytes(const sbp_ctx* c) { return c->tf_on ? (2 * (size_t)c->tf_len + 1) * sizeof(double) : 0; }

// grid type per component and axis: true = "+" (n+1 nodes), false = "-" (n+2), Table T1
const bool kPlus[6][3] = {{false, true, true}, {true, false, true}, {true, true, false},
                          {true, false, false}, {false, true, false}, {false, false, true}};

int comp_dim(const HostBlock& b, int c, int a) { return kPlus[c][a] ? b.n[a] + 1 : b.n[a] + 2; }

// ---------------------------------------------------------- closure tables
// Appendix rows (times h): D+ rows 0, 1, n-1, n; D- rows 0, 1, 2, n-1, n, n+1.
// SAT row changes (Section III): a PEC face flips the boundary-E coefficient
// of the D- face row (H update), a PMC or absorbing face flips the boundary-H
// coefficient of the D+ face row (E update); an interface face moves that
// coefficient onto the neighbour's value (penalties of EPBC1-6 at zero phase
// with sigma = chi = +-1/2).
Row mkrow(int s, double c0, double c1, double c2, double ih) {
  Row r;
  r.s = s;
  r.nbr = 0;
  r.c[0] = c0 * ih;
  r.c[1] = c1 * ih;
  r.c[2] = c2 * ih;
  r.cn = 0.0;
  return r;
}

// Convolutional PML profiles of a block: for axis a, grid g ("+" 0, "-" 1)
// and quantity q (0: b, 1: c, 2: 1/kappa), P entries per node index (the
// "+" grid's node n+1 and any index past the grid are neutral: 1, 0, 1).
// At depth rho in [0, 1] into a layer of `cells` cells next to a face set to
// SBP_CPML: sigma = sigma_max rho^m with sigma_max = sigma_factor (m+1) /
// (eta0 h), kappa = 1 + (kappa_max - 1) rho^m, alpha = alpha_max (1 - rho);
// b = exp(-(sigma/kappa + alpha) dt/eps0), c = sigma (b-1) / (sigma kappa +
// kappa^2 alpha).  Node positions: "+" grid i h, "-" grid 0, (j-1/2) h, n h.
void pml_profiles(const sbp_ctx* c, const HostBlock& b, int P, std::vector<double>& out) {
  const double eta0 = std::sqrt(kMu0 / kEps0);
  for (int a = 0; a < 3; ++a) {
    const int n = b.n[a];
    const double h = b.h[a], L = n * h;
    const bool lo = b.iface[2 * a] < 0 && b.faces[2 * a] == SBP_CPML;
    const bool hi = b.iface[2 * a + 1] < 0 && b.faces[2 * a + 1] == SBP_CPML;
    const double d = c->pml_cells * h;
    const double smax = c->pml_sigma_factor * (c->pml_m + 1) / (eta0 * h);
    for (int g = 0; g < 2; ++g) {
      std::vector<double> vb(P, 1.0), vc(P, 0.0), vk(P, 1.0);
      const int cnt = g == 0 ? n + 1 : n + 2;
      for (int idx = 0; idx < cnt; ++idx) {
        const double x = g == 0 ? idx * h : (idx == 0 ? 0.0 : (idx == n + 1 ? L : (idx - 0.5) * h));
        double rho = 0.0;
        if (lo) rho = std::max(rho, std::min(std::max((d - x) / d, 0.0), 1.0));
        if (hi) rho = std::max(rho, std::min(std::max((x - (L - d)) / d, 0.0), 1.0));
        if (rho <= 0.0) continue;
        const double rm = std::pow(rho, c->pml_m);
        const double sig = smax * rm, kap = 1.0 + (c->pml_kappa_max - 1.0) * rm;
        const double alp = c->pml_alpha_max * (1.0 - rho);
        const double bb = std::exp(-(sig / kap + alp) * c->dt / kEps0);
        const double den = sig * kap + kap * kap * alp;
        vb[idx] = bb;
        vc[idx] = sig > 0.0 ? sig * (bb - 1.0) / den : 0.0;
        vk[idx] = 1.0 / kap;
      }
      out.insert(out.end(), vb.begin(), vb.end());
      out.insert(out.end(), vc.begin(), vc.end());
      out.insert(out.end(), vk.begin(), vk.end());
    }
  }
}

void build_rows(const HostBlock& b, DevBlock& d) {
  for (int a = 0; a < 3; ++a) {
    const int n = b.n[a];
    const double ih = 1.0 / b.h[a];
    const int flo = b.faces[2 * a], fhi = b.faces[2 * a + 1];
    const bool ilo = b.iface[2 * a] >= 0, ihi = b.iface[2 * a + 1] >= 0;
    (void)n;
    // D+ (E update)
    d.dp[a][0] = mkrow(0, -1.0, 0.5, 0.5, ih);
    d.dp[a][1] = mkrow(-1, -0.5, -0.25, 0.75, ih);
    d.dp[a][2] = mkrow(0, -0.75, 0.25, 0.5, ih);
    d.dp[a][3] = mkrow(-1, -0.5, -0.5, 1.0, ih);
    if (ilo) {
      d.dp[a][0].cn = d.dp[a][0].c[0];
      d.dp[a][0].c[0] = 0.0;
      d.dp[a][0].nbr = 1;
    } else if (flo == SBP_PMC || flo == SBP_ABC1) {
      d.dp[a][0].c[0] = -d.dp[a][0].c[0];
    }
    if (ihi) {
      d.dp[a][3].cn = d.dp[a][3].c[2];
      d.dp[a][3].c[2] = 0.0;
      d.dp[a][3].nbr = 1;
    } else if (fhi == SBP_PMC || fhi == SBP_ABC1) {
      d.dp[a][3].c[2] = -d.dp[a][3].c[2];
    }
    // D- (H update)
    d.dm[a][0] = mkrow(0, -1.0, 1.0, 0.0, ih);
    d.dm[a][1] = mkrow(-1, -1.0, 1.0, 0.0, ih);
    d.dm[a][2] = mkrow(-2, -0.2, -0.6, 0.8, ih);
    d.dm[a][3] = mkrow(-1, -0.8, 0.6, 0.2, ih);
    d.dm[a][4] = mkrow(-2, 0.0, -1.0, 1.0, ih);
    d.dm[a][5] = mkrow(-3, 0.0, -1.0, 1.0, ih);
    if (ilo) {
      d.dm[a][0].cn = d.dm[a][0].c[0];
      d.dm[a][0].c[0] = 0.0;
      d.dm[a][0].nbr = 1;
    } else if (flo == SBP_PEC || flo == SBP_CPML) {  // a PEC face behind an absorbing layer
      d.dm[a][0].c[0] = -d.dm[a][0].c[0];
    }
    if (ihi) {
      d.dm[a][5].cn = d.dm[a][5].c[2];
      d.dm[a][5].c[2] = 0.0;
      d.dm[a][5].nbr = 1;
    } else if (fhi == SBP_PEC || fhi == SBP_CPML) {
      d.dm[a][5].c[2] = -d.dm[a][5].c[2];
    }
  }
}

// ------------------------------------------------ 1:2 interface operators
// Node coordinates (units of the coarse h) and norm weights of the two 1D
// grids (Section II-A, Appendix).
std::vector<double> nodes(bool plus, int n, double h) {
  std::vector<double> x;
  if (plus) {
    for (int i = 0; i <= n; ++i) x.push_back(i * h);
  } else {
    x.push_back(0.0);
    for (int j = 1; j <= n; ++j) x.push_back((j - 0.5) * h);
    x.push_back(n * h);
  }
  return x;
}
std::vector<double> norm_weights(bool plus, int n, double h) {
  std::vector<double> w;
  if (plus) {
    for (int i = 0; i <= n; ++i) w.push_back((i == 0 || i == n) ? 0.5 * h : h);
  } else {
    for (int r = 0; r <= n + 1; ++r) {
      double v = 1.0;
      if (r == 0 || r == n + 1) v = 0.5;
      else if (r == 1 || r == n) v = 0.25;
      else if (r == 2 || r == n - 1) v = 1.25;
      w.push_back(v * h);
    }
  }
  return w;
}

// Coarse-to-fine interpolation, dense (rows = fine nodes).  "+" grid: linear
// interpolation (fine nodes at coarse nodes and midpoints).  "-" grid:
// linear interpolation inside; the four fine rows at each end, over the
// first three coarse nodes, are the rows nearest (Frobenius) to linear
// interpolation such that every row sums to one and the fine-norm-weighted
// column sums equal the coarse norm weights (the restriction
// Wc^-1 I^T Wf then reproduces constants).  Exact values of that solution:
const double kMinusBlock[4][3] = {{49.0 / 46, -13.0 / 92, 7.0 / 92},
                                  {49.0 / 92, 79.0 / 184, 7.0 / 184},
                                  {15.0 / 92, 73.0 / 184, 81.0 / 184},
                                  {3.0 / 23, -3.0 / 92, 83.0 / 92}};

std::vector<double> c2f(bool plus, int nc) {
  const std::vector<double> xc = nodes(plus, nc, 1.0), xf = nodes(plus, 2 * nc, 0.5);
  const int rf = (int)xf.size(), rc = (int)xc.size();
  std::vector<double> m((size_t)rf * rc, 0.0);
  for (int r = 0; r < rf; ++r) {
    int i = 0;
    while (i + 2 < rc && xc[i + 1] <= xf[r]) ++i;
    const double t = (xf[r] - xc[i]) / (xc[i + 1] - xc[i]);
    m[(size_t)r * rc + i] = 1.0 - t;
    m[(size_t)r * rc + i + 1] = t;
  }
  if (!plus) {
    for (int r = 0; r < 4; ++r)
      for (int s = 0; s < rc; ++s) {
        m[(size_t)r * rc + s] = s < 3 ? kMinusBlock[r][s] : 0.0;
        m[(size_t)(rf - 1 - r) * rc + s] = s >= rc - 3 ? kMinusBlock[r][rc - 1 - s] : 0.0;
      }
  }
  return m;
}

// rows of a dense matrix as tap lists (consecutive support)
bool to_taps(const std::vector<double>& m, int rows, int cols, std::vector<Taps>& out) {
  for (int r = 0; r < rows; ++r) {
    int lo = cols, hi = -1;
    for (int c = 0; c < cols; ++c)
      if (m[(size_t)r * cols + c] != 0.0) {
        lo = std::min(lo, c);
        hi = std::max(hi, c);
      }
    Taps t;
    std::memset(&t, 0, sizeof(t));
    if (hi < lo) {
      t.start = 0;
      t.count = 0;
    } else {
      if (hi - lo + 1 > MAX_TAPS) return false;
      t.start = lo;
      t.count = hi - lo + 1;
      for (int c = lo; c <= hi; ++c) t.w[c - lo] = m[(size_t)r * cols + c];
    }
    out.push_back(t);
  }
  return true;
}

// taps mapping neighbour nodes to own nodes along one tangential axis
bool axis_taps(bool plus, int own_n, int role, std::vector<Taps>& out) {
  if (role == 0) {  // same mesh
    const int cnt = plus ? own_n + 1 : own_n + 2;
    for (int r = 0; r < cnt; ++r) {
      Taps t;
      std::memset(&t, 0, sizeof(t));
      t.start = r;
      t.count = 1;
      t.w[0] = 1.0;
      out.push_back(t);
    }
    return true;
  }
  if (role == 1) {  // own fine, neighbour coarse: I_c2f
    const int nc = own_n / 2;
    const std::vector<double> m = c2f(plus, nc);
    return to_taps(m, plus ? 2 * nc + 1 : 2 * nc + 2, plus ? nc + 1 : nc + 2, out);
  }
  // own coarse, neighbour fine: I_f2c = Wc^-1 I_c2f^T Wf
  const int nc = own_n;
  const std::vector<double> m = c2f(plus, nc);
  const int rf = plus ? 2 * nc + 1 : 2 * nc + 2, rc = plus ? nc + 1 : nc + 2;
  const std::vector<double> wc = norm_weights(plus, nc, 1.0), wf = norm_weights(plus, 2 * nc, 0.5);
  std::vector<double> r((size_t)rc * rf, 0.0);
  for (int i = 0; i < rc; ++i)
    for (int f = 0; f < rf; ++f) r[(size_t)i * rf + f] = m[(size_t)f * rc + i] * wf[f] / wc[i];
  return to_taps(r, rc, rf, out);
}

template <typename T>
void put_cells(std::vector<T>& dst, size_t off, const std::vector<double>& src) {
  for (size_t q = 0; q < src.size(); ++q) dst[off + q] = (T)src[q];
}

// A block's per-cell permittivity as byte indices into a table of at most
// kCellTab values in the field precision (the very values the kernels would
// read from the cell array, so results are unchanged); false if the cells
// take more values.
template <typename T>
bool table_cells(const std::vector<double>& eps, unsigned char* idx, T* tab) {
  int n = 0, li = -1;
  T last = T(0);
  for (size_t q = 0; q < eps.size(); ++q) {
    const T v = (T)eps[q];
    if (li < 0 || v != last) {
      li = -1;
      for (int e = 0; e < n && li < 0; ++e)
        if (tab[e] == v) li = e;
      if (li < 0) {
        if (n == kCellTab) return false;
        tab[n] = v;
        li = n++;
      }
      last = v;
    }
    idx[q] = (unsigned char)li;
  }
  return true;
}

template <typename T>
sbp_status upload_tables(sbp_ctx* c) {
  const size_t nb = c->blocks.size();
  std::vector<unsigned char> idx;
  std::vector<T> tab(nb * kCellTab, T(1));
  bool any = false;
  size_t off = 0;
  for (size_t bi = 0; bi < nb; ++bi) {
    HostBlock& b = c->blocks[bi];
    b.tabled = false;
    if (!b.eps.empty() && !c->tables_off) {
      if (idx.empty()) idx.assign(c->ncells, 0);
      b.tabled = table_cells<T>(b.eps, idx.data() + off, tab.data() + bi * kCellTab);
      any = any || b.tabled;
    }
    off += (size_t)b.n[0] * b.n[1] * b.n[2];
  }
  if (!any) return SBP_OK;
  if (!c->d_midx) {
    c->d_midx = (unsigned char*)dalloc(c, c->ncells);
    if (!c->d_midx) return fail(c, SBP_ENOMEM, "material allocation failed");
  }
  if (!c->d_mtab) {
    c->d_mtab = dalloc(c, nb * kCellTab * sizeof(T));
    if (!c->d_mtab) return fail(c, SBP_ENOMEM, "material allocation failed");
    c->mtab_blocks = nb;
  }
  HIPCHK(c, hipMemcpyAsync(c->d_midx, idx.data(), idx.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_mtab, tab.data(), tab.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SBP_OK;
}

sbp_status upload_materials(sbp_ctx* c) {
  const bool fp64 = c->prec == SBP_FP64;
  for (int kind = 0; kind < 3; ++kind) {
    bool any = false;
    for (auto& b : c->blocks) {
      const std::vector<double>& v = kind == 0 ? b.eps : (kind == 1 ? b.mu : b.sig);
      any |= !v.empty();
    }
    if (!any) continue;
    if (!c->mat[kind]) {
      c->mat[kind] = dalloc(c, c->ncells * elem_size(c));
      if (!c->mat[kind]) return fail(c, SBP_ENOMEM, "material allocation failed");
    }
    std::vector<double> dflt;
    if (fp64) {
      std::vector<double> h(c->ncells, kind == 2 ? 0.0 : 1.0);
      size_t off = 0;
      for (auto& b : c->blocks) {
        const std::vector<double>& v = kind == 0 ? b.eps : (kind == 1 ? b.mu : b.sig);
        if (!v.empty()) put_cells(h, off, v);
        off += (size_t)b.n[0] * b.n[1] * b.n[2];
      }
      HIPCHK(c, hipMemcpyAsync(c->mat[kind], h.data(), h.size() * 8, hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
      std::vector<float> h(c->ncells, kind == 2 ? 0.0f : 1.0f);
      size_t off = 0;
      for (auto& b : c->blocks) {
        const std::vector<double>& v = kind == 0 ? b.eps : (kind == 1 ? b.mu : b.sig);
        if (!v.empty()) put_cells(h, off, v);
        off += (size_t)b.n[0] * b.n[1] * b.n[2];
      }
      HIPCHK(c, hipMemcpyAsync(c->mat[kind], h.data(), h.size() * 4, hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
  }
  const sbp_status ts = fp64 ? upload_tables<double>(c) : upload_tables<float>(c);
  if (ts != SBP_OK) return ts;
  // flags per block
  for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
    const HostBlock& b = c->blocks[bi];
    DevBlock& d = c->hblocks[bi];
    d.mat = (b.eps.empty() ? 0 : MAT_EPS) | (b.mu.empty() ? 0 : MAT_MU) | (b.sig.empty() ? 0 : MAT_SIG);
  }
  HIPCHK(c, hipMemcpyAsync(c->d_blocks, c->hblocks.data(), c->hblocks.size() * sizeof(DevBlock),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return SBP_OK;
}

void drop_graph(sbp_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}

int round8(size_t v) { return (int)((v + 7) / 8 * 8); }

// Workgroups of a step launch: one per tile (or the resident count set by
// sbp_set_launch), rounded up to a multiple of the 8 XCDs so the kernels can
// hand each XCD a contiguous range of tiles.
int grid_of(const sbp_ctx* c, int ntiles) {
  const int g = c->wgs > 0 ? std::min(c->wgs, ntiles) : ntiles;
  return round8((size_t)std::max(g, 1));
}

// Kind of a block for the step kernels: bit 0 = per-cell permittivity,
// bit 1 = general (conductivity, absorbing faces, per-cell permeability,
// absorbing layers or the TF/SF box), bit 2 = interface or periodic faces
// (the interface rows are compiled only into those variants; without bit 1
// the loss and absorbing terms are left out), bit 3 = CPML layers, bit 4 =
// the TF/SF box (its corrections are compiled only into that variant);
// plain PEC/PMC blocks take the lean kernels.
bool has_pml(const HostBlock& b) {
  for (int f = 0; f < 6; ++f)
    if (b.iface[f] < 0 && b.faces[f] == SBP_CPML) return true;
  return false;
}

int block_kind(const HostBlock& b) {
  bool gen = !b.mu.empty() || !b.sig.empty(), iface = false;
  for (int f = 0; f < 6; ++f) {
    iface = iface || b.iface[f] >= 0;
    gen = gen || b.faces[f] == SBP_ABC1;
  }
  const bool pml = has_pml(b);
  gen = gen || b.tfsf;
  return (b.eps.empty() ? 0 : 1) | (gen || pml ? 2 : 0) | (iface ? 4 : 0) | (pml ? 8 : 0) | (b.tfsf ? 16 : 0);
}

// Windows of W node columns along an axis of s = n+2 nodes for the one-pass
// step: window t starts at st[t] and owns [lo[t], hi[t]]; all but the last
// own W-1 columns (the last column of a window only supplies neighbour values
// of H); the last window is moved back to end at the box edge and owns from
// n-1 at the latest, so that the D+ closure rows of the far face (which reach
// up to node n+1) lie inside one window.
void windows(int s, int n, int W, std::vector<int>& st, std::vector<int>& lo, std::vector<int>& hi) {
  if (s <= W) {
    st = {0};
    lo = {0};
    hi = {s - 1};
    return;
  }
  const int T = (s + W - 2) / (W - 1);
  st.resize(T);
  lo.resize(T);
  hi.resize(T);
  for (int t = 0; t < T; ++t) {
    st[t] = t < T - 1 ? (W - 1) * t : s - W;
    lo[t] = t < T - 1 ? (W - 1) * t : std::min((W - 1) * (T - 1), n - 1);
  }
  for (int t = 0; t < T; ++t) hi[t] = t < T - 1 ? lo[t + 1] - 1 : s - 1;
}

// Whether a tile of the TF/SF block holds a node that the box surface
// couples across (bit 2 of the tile flags): such nodes have all indices in
// [lo-1, hi+1] and one of them in {lo-1, lo, hi, hi+1}.
bool tf_tile(const sbp_ctx* c, long long sx, long long q0, int threads, int z0, int cz, long long sxy) {
  const int* bx = c->tf_box;
  auto near = [&](int v, int a) { return v >= bx[2 * a] - 1 && v <= bx[2 * a + 1] + 1; };
  auto edge = [&](int v, int a) { return v <= bx[2 * a] || v >= bx[2 * a + 1]; };
  const long long q1 = std::min<long long>(q0 + threads, sxy);
  for (int k = z0; k < z0 + cz; ++k) {
    if (!near(k, 2)) continue;
    for (long long q = q0; q < q1; ++q) {
      const int j = (int)(q / sx), i = (int)(q - j * sx);
      if (near(i, 0) && near(j, 1) && (edge(i, 0) || edge(j, 1) || edge(k, 2))) return true;
    }
  }
  return false;
}

sbp_status build_tiles(sbp_ctx* c) {
  std::vector<Tile> tl;
  c->near_dirty = true;
  const int threads = c->tx * c->ty;
  // lossless interface blocks take the lean interface kernels unless another
  // block needs the general interface ones: then they join that kind, so that
  // a half step stays one launch (two back-to-back launches cost more than
  // the general terms the lossless blocks skip at run time)
  // Plain blocks with a permittivity table take the tabled E kernel (kind
  // bit 5) with one workgroup per tile of at least 8 planes: measured on the
  // 256^3 dielectric block, the E launch gains 1.5% there, and loses 2.5%
  // at 4 planes per tile and 17% with resident workgroups (2048 x 128
  // threads), where the byte loads and table reads cost more than the bytes
  // they save.
  const bool tables = c->wgs == 0 && c->cz >= 8;
  bool gen_iface = false;
  for (const HostBlock& b : c->blocks) gen_iface = gen_iface || (block_kind(b) & 6) == 6;
  auto kind_of = [&](const HostBlock& b) {
    const int k = block_kind(b);
    if (k == 1 && b.tabled && tables) return k | 32;
    return (gen_iface && (k & 30) == 4) ? (k | 2) : k;
  };
  for (int kind : kKindOrder.k) {
    c->kind_t0[kind] = (int)tl.size();
    for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
      const HostBlock& b = c->blocks[bi];
      if (kind_of(b) != kind) continue;
      const long long sx = b.n[0] + 2, sxy = sx * (b.n[1] + 2);
      for (int z0 = 0; z0 < b.n[2] + 2; z0 += c->cz)
        for (long long q0 = 0; q0 < sxy; q0 += threads) {
          // flags: bit 0 = a source, bit 1 = a probe lies in the tile
          int flags = 0;
          auto inside = [&](int i, int j, int k) {
            const long long q = i + sx * j;
            return q >= q0 && q < q0 + threads && k >= z0 && k < z0 + c->cz;
          };
          for (auto& sr : c->srcs)
            if (sr.block == (int)bi && inside(sr.s.i, sr.s.j, sr.s.k)) flags |= 1;
          for (auto& pr : c->prbs)
            if (pr.block == (int)bi && inside(pr.p.i, pr.p.j, pr.p.k)) flags |= 2;
          if (b.tfsf && tf_tile(c, sx, q0, threads, z0, c->cz, sxy)) flags |= 4;
          tl.push_back(Tile{(int)bi, (int)q0, z0, flags});
        }
    }
    c->kind_t1[kind] = (int)tl.size();
  }
  if (tl.size() > c->tiles_cap) {
    dfree(c, c->d_tiles);
    c->d_tiles = (Tile*)dalloc(c, tl.size() * sizeof(Tile));
    if (!c->d_tiles) return fail(c, SBP_ENOMEM, "tile list allocation failed");
    c->tiles_cap = tl.size();
  }
  c->ntiles = (int)tl.size();
  HIPCHK(c, hipMemcpyAsync(c->d_tiles, tl.data(), tl.size() * sizeof(Tile), hipMemcpyHostToDevice, c->stream));
  // the same tiles without source / probe flags, for the adjoint state
  if (tl.size() > c->bare_cap) {
    dfree(c, c->d_tiles_bare);
    c->d_tiles_bare = (Tile*)dalloc(c, tl.size() * sizeof(Tile));
    if (!c->d_tiles_bare) return fail(c, SBP_ENOMEM, "tile list allocation failed");
    c->bare_cap = tl.size();
  }
  c->bare.assign(tl.begin(), tl.end());
  for (Tile& t : c->bare) t.pad = 0;
  HIPCHK(c, hipMemcpyAsync(c->d_tiles_bare, c->bare.data(), c->bare.size() * sizeof(Tile), hipMemcpyHostToDevice,
                           c->stream));
  // one-pass tiles of the plain kinds
  std::vector<FTile> ft;
  for (int kind = 0; kind < 2; ++kind) {
    c->fk_t0[kind] = (int)ft.size();
    for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
      const HostBlock& b = c->blocks[bi];
      if (block_kind(b) != kind) continue;  // the one-pass kernel reads the cells themselves
      std::vector<int> xs, xl, xh, ys, yl, yh, zl, zh;
      windows(b.n[0] + 2, b.n[0], FX, xs, xl, xh);
      windows(b.n[1] + 2, b.n[1], FY, ys, yl, yh);
      for (int z = 0; z == 0 || z < b.n[2] - 1; z += c->fz) zl.push_back(z);
      for (size_t q = 0; q < zl.size(); ++q) zh.push_back(q + 1 < zl.size() ? zl[q + 1] - 1 : b.n[2] + 1);
      for (size_t zq = 0; zq < zl.size(); ++zq)
        for (size_t yq = 0; yq < ys.size(); ++yq)
          for (size_t xq = 0; xq < xs.size(); ++xq) {
            FTile f{(int)bi, xs[xq], ys[yq], xl[xq], xh[xq], yl[yq], yh[yq], zl[zq], zh[zq], 0};
            auto inside = [&](int i, int j, int k) {
              return i >= f.olx && i <= f.ohx && j >= f.oly && j <= f.ohy && k >= f.z0 && k <= f.z1;
            };
            for (auto& sr : c->srcs)
              if (sr.block == (int)bi && inside(sr.s.i, sr.s.j, sr.s.k)) f.flags |= 1;
            for (auto& pr : c->prbs)
              if (pr.block == (int)bi && inside(pr.p.i, pr.p.j, pr.p.k)) f.flags |= 2;
            ft.push_back(f);
          }
    }
    c->fk_t1[kind] = (int)ft.size();
  }
  if (ft.size() > c->ftiles_cap) {
    dfree(c, c->d_ftiles);
    dfree(c, c->d_ftiles_bare);
    c->d_ftiles = (FTile*)dalloc(c, ft.size() * sizeof(FTile));
    c->d_ftiles_bare = (FTile*)dalloc(c, ft.size() * sizeof(FTile));
    if (!c->d_ftiles || !c->d_ftiles_bare) return fail(c, SBP_ENOMEM, "tile list allocation failed");
    c->ftiles_cap = ft.size();
  }
  if (!ft.empty()) {
    HIPCHK(c, hipMemcpyAsync(c->d_ftiles, ft.data(), ft.size() * sizeof(FTile), hipMemcpyHostToDevice, c->stream));
    c->fbare.assign(ft.begin(), ft.end());
    for (FTile& f : c->fbare) f.flags = 0;
    HIPCHK(c, hipMemcpyAsync(c->d_ftiles_bare, c->fbare.data(), ft.size() * sizeof(FTile), hipMemcpyHostToDevice,
                             c->stream));
  }
  size_t sum = 0;
  for (int kind : kKindOrder.k)
    if (c->kind_t1[kind] > c->kind_t0[kind]) sum += (size_t)grid_of(c, c->kind_t1[kind] - c->kind_t0[kind]);
  size_t fsum = 0;
  for (int kind = 0; kind < 2; ++kind)
    if (c->fk_t1[kind] > c->fk_t0[kind]) fsum += (size_t)grid_of(c, c->fk_t1[kind] - c->fk_t0[kind]);
  const size_t grid = 2 * sum + fsum + 8;  // partial sums of all launches of a step
  c->partials_need = grid;
  if (grid > c->partials_cap) {
    dfree(c, c->d_partials);
    c->d_partials = (double*)dalloc(c, grid * sizeof(double));
    if (!c->d_partials) return fail(c, SBP_ENOMEM, "partials allocation failed");
    c->partials_cap = grid;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  return SBP_OK;
}

// Tile walk of the step kernels: contiguous ranges per XCD when the fields
// and materials fit in the eight XCDs' L2 caches together (8 x 4 MB), so
// each XCD's share stays resident from step to step; grouped dispatch order
// otherwise (the step streams through the Infinity Cache or HBM).
int tile_order(const sbp_ctx* c) {
  size_t bytes = c->pool_elems * elem_size(c);
  for (int m = 0; m < 3; ++m)
    if (c->mat[m]) bytes += c->ncells * elem_size(c);
  return bytes > (size_t(32) << 20) ? 0 : 1;
}

KArgs kargs(sbp_ctx* c) {
  KArgs a;
  a.blocks = c->d_blocks;
  a.tiles = c->d_tiles;
  a.ftiles = c->d_ftiles;
  a.ntiles = c->ntiles;
  a.cz = c->cz;
  a.order = tile_order(c);
  a.hpoff = -1;
  a.pool = c->pool;
  a.pool2 = c->pool2;
  a.mat_eps = c->mat[0];
  a.mat_idx = c->d_midx;
  a.mat_tab = c->d_mtab;
  a.mat_mu = c->mat[1];
  a.mat_sig = c->mat[2];
  a.face = c->d_face;
  a.pml_prof = c->d_pml;
  a.psi = c->d_psi;
  a.src = c->d_src;
  a.srcval = c->d_srcval;
  a.nsrc = c->nsrc_total;
  a.prb = c->d_prb;
  a.energy = c->d_energy;
  a.ecap = (int)c->history;
  a.probes = c->d_probes;
  a.pcap = (int)c->history;
  a.partials = c->d_partials;
  a.st = c->d_st;
  a.dt = c->dt;
  a.eps0 = kEps0;
  a.mu0 = kMu0;
  a.nblocks = (int)c->blocks.size();
  a.t0 = 0;
  a.t1 = c->ntiles;
  a.poff = 0;
  a.tf = c->tf_on ? c->d_tf : nullptr;
  return a;
}

// The pool holding the state (E^n, H^{n-1/2}) at step n.
void* pool_at(const sbp_ctx* c, long long n) { return (n & 1) ? c->pool2 : c->pool; }


// One leapfrog step: [gather E faces] -> H update -> [gather H faces] -> E
// update, each update one launch per block kind.  The H workgroups write the
// H part of W^n per tile, the E workgroups add the E part (from E^n) and the
// same tile's H partial, and the finish kernel sums the E partials into
// energy slot n and advances the step index.
// One leapfrog step of the state that `a` points at (pool, face buffers,
// energy / probe rings, step counter): the forward state (kargs(c)) or the
// adjoint state of sbp_adjoint.
// Tile ranges per kind and gather workgroup tables of a step over part of
// the blocks (local time stepping); null: the context's own.
struct StepLists {
  const int *kt0, *kt1;
  const GatherWG *wg_e, *wg_h;
  int nwg_e, nwg_h;
  bool finish;  // false: no finish kernel (no energy, step index or sources)
};

sbp_status enqueue_step_on(sbp_ctx* c, KArgs a, bool events, const StepLists* lists = nullptr) {
  const int threads = c->tx * c->ty;
  const int* kt0 = lists ? lists->kt0 : c->kind_t0;
  const int* kt1 = lists ? lists->kt1 : c->kind_t1;
  const GatherWG* wg_e = lists ? lists->wg_e : c->d_wg_e;
  const GatherWG* wg_h = lists ? lists->wg_h : c->d_wg_h;
  const int nwg_e = lists ? lists->nwg_e : c->nwg_e, nwg_h = lists ? lists->nwg_h : c->nwg_h;
  const bool f64 = c->prec == SBP_FP64;
  hipError_t e;
  double* face = const_cast<double*>(a.face);
  auto mark = [&]() -> sbp_status {
    if (events) HIPCHK(c, hipEventRecord(c->kev[c->kev_used++], c->stream));
    return SBP_OK;
  };
  // kinds stepped by the two-pass kernels: all, or only the general ones
  auto two_pass = [&](int kind) { return kt1[kind] > kt0[kind] && (!c->fused || (kind & 6)); };
  if (c->njobs_e) {
    e = f64 ? launch_gather<double>(c->d_blocks, c->d_jobs_e, wg_e, nwg_e, c->d_taps, a, 0, face, c->stream)
            : launch_gather<float>(c->d_blocks, c->d_jobs_e, wg_e, nwg_e, c->d_taps, a, 0, face, c->stream);
    HIPCHK(c, e);
  }
  sbp_status st = mark();
  if (st != SBP_OK) return st;
  // partial sums: the H launches write slots [0, nh); each E workgroup adds
  // the H partial of its tile (same tile list and grid) to its own, so the
  // finish sums the E and one-pass slots [nh, nparts) only
  int nparts = 0, hpoff[kKinds];
  for (int& v : hpoff) v = -1;
  a.hpoff = -1;
  for (int kind : kKindOrder.k) {
    if (!two_pass(kind)) continue;
    a.t0 = kt0[kind];
    a.t1 = kt1[kind];
    a.poff = hpoff[kind] = nparts;
    const int grid = grid_of(c, a.t1 - a.t0);
    nparts += grid;
    e = f64 ? launch_h<double>(a, kind, grid, threads, c->stream) : launch_h<float>(a, kind, grid, threads, c->stream);
    HIPCHK(c, e);
  }
  const int nh = nparts;
  if ((st = mark()) != SBP_OK) return st;
  if (c->njobs_h) {
    e = f64 ? launch_gather<double>(c->d_blocks, c->d_jobs_h, wg_h, nwg_h, c->d_taps, a, 1, face, c->stream)
            : launch_gather<float>(c->d_blocks, c->d_jobs_h, wg_h, nwg_h, c->d_taps, a, 1, face, c->stream);
    HIPCHK(c, e);
  }
  if ((st = mark()) != SBP_OK) return st;
  for (int kind : kKindOrder.k) {
    if (!two_pass(kind)) continue;
    a.t0 = kt0[kind];
    a.t1 = kt1[kind];
    a.poff = nparts;
    a.hpoff = hpoff[kind];
    const int grid = grid_of(c, a.t1 - a.t0);
    nparts += grid;
    e = f64 ? launch_e<double>(a, kind, grid, threads, c->stream) : launch_e<float>(a, kind, grid, threads, c->stream);
    HIPCHK(c, e);
  }
  a.hpoff = -1;
  if ((st = mark()) != SBP_OK) return st;
  if ((st = mark()) != SBP_OK) return st;
  if (c->fused) {
    for (int kind = 0; kind < 2; ++kind) {
      if (c->fk_t1[kind] == c->fk_t0[kind]) continue;
      a.t0 = c->fk_t0[kind];
      a.t1 = c->fk_t1[kind];
      a.poff = nparts;
      const int grid = grid_of(c, a.t1 - a.t0);
      nparts += grid;
      e = f64 ? launch_fused<double>(a, kind, grid, c->stream) : launch_fused<float>(a, kind, grid, c->stream);
      HIPCHK(c, e);
    }
  }
  if ((st = mark()) != SBP_OK) return st;
  if (lists && !lists->finish) return SBP_OK;
  HIPCHK(c, launch_finish(a, nh, nparts, c->stream));  // W^n into ring slot n; n += 1; sources of step n+1
  return SBP_OK;
}

sbp_status enqueue_step(sbp_ctx* c, bool events) { return enqueue_step_on(c, kargs(c), events); }

bool check_block(const sbp_ctx* c, int b) { return b >= 0 && b < (int)c->blocks.size(); }

template <typename T>
void extract(const std::vector<T>& box, const DevBlock& d, const int s[3], double* dst) {
  size_t q = 0;
  for (int k = 0; k < s[2]; ++k)
    for (int j = 0; j < s[1]; ++j)
      for (int i = 0; i < s[0]; ++i) dst[q++] = (double)box[(size_t)i + d.sx * j + d.sxy * k];
}
template <typename T>
void insert(std::vector<T>& box, const DevBlock& d, const int s[3], const double* src) {
  size_t q = 0;
  for (int k = 0; k < s[2]; ++k)
    for (int j = 0; j < s[1]; ++j)
      for (int i = 0; i < s[0]; ++i) box[(size_t)i + d.sx * j + d.sxy * k] = (T)src[q++];
}

// L u of local time stepping: one step with unit time step of the scratch
// state (E = u, H = 0, prepared in lts_s) with its own face buffers, step
// counter and energy ring, on the tiles that meet the near boxes (all tiles:
// `whole`), without source / probe flags: the E part afterwards holds
// u - L u there.
sbp_status lts_apply(sbp_ctx* c, bool whole) {
  KArgs a = kargs(c);
  a.blocks = c->lts_blocks;
  a.pool = a.pool2 = c->lts_s;
  a.face = c->lts_face;
  a.st = c->lts_st;
  a.energy = a.probes = c->lts_ring;
  a.ecap = a.pcap = 1;
  a.tiles = whole ? c->d_tiles_bare : c->d_near;
  a.ftiles = c->d_ftiles_bare;
  a.nsrc = 0;
  a.dt = 1.0;
  a.tf = nullptr;
  if (whole) return enqueue_step_on(c, a, false);
  const StepLists near{c->nk_t0, c->nk_t1, c->d_nwg[0], c->d_nwg[1], c->nnwg[0], c->nnwg[1], false};
  return enqueue_step_on(c, a, false, &near);
}

// Boxes of local time stepping: a refined block whole; in another block the
// nodes within `reach` of its own cells of a refined block's box (the
// bounding box over the refined blocks).  The near boxes (reach 2) hold
// every E node where the scheme's E^{n+1} differs from the ordinary step's
// (those within one cell); the operator's tiles meet the wider boxes
// (reach 4), so that the H and E values the near boxes read (one cell
// farther each) are formed from nonzero input.
constexpr int kLtsNear = 2, kLtsWide = 4;
std::vector<LtsBox> lts_boxes(const sbp_ctx* c, const std::vector<int>& refined, int reach) {
  const int nb = (int)c->blocks.size();
  std::vector<LtsBox> out(nb, LtsBox{{0, 0, 0}, {-1, -1, -1}, 0, 0});
  for (int y = 0; y < nb; ++y) {
    const HostBlock& Y = c->blocks[y];
    LtsBox& bx = out[y];
    if (refined[y]) {
      for (int a = 0; a < 3; ++a) {
        bx.lo[a] = 0;
        bx.hi[a] = Y.n[a] + 1;
      }
      bx.on = bx.refined = 1;
      continue;
    }
    for (int f = 0; f < nb; ++f) {
      if (!refined[f]) continue;
      const HostBlock& F = c->blocks[f];
      int lo[3], hi[3];
      bool hit = true;
      for (int a = 0; a < 3 && hit; ++a) {
        const double h = Y.h[a], tol = 1e-9 * h;
        const double flo = F.x0[a] - reach * h, fhi = F.x0[a] + F.n[a] * F.h[a] + reach * h;
        const double ylo = Y.x0[a], yhi = Y.x0[a] + Y.n[a] * h;
        const double l = std::max(flo, ylo), u = std::min(fhi, yhi);
        if (l > u + tol) {
          hit = false;
          break;
        }
        // cells [cl, cu] of Y meet the interval; their nodes, with one more
        // on each side for the "-" grid's half-cell offsets
        const int cl = (int)std::floor((l - ylo) / h + 1e-9), cu = (int)std::ceil((u - ylo) / h - 1e-9);
        lo[a] = std::max(0, cl - 1);
        hi[a] = std::min(Y.n[a] + 1, cu + 1);
      }
      if (!hit) continue;
      for (int a = 0; a < 3; ++a) {
        bx.lo[a] = bx.on ? std::min(bx.lo[a], lo[a]) : lo[a];
        bx.hi[a] = bx.on ? std::max(bx.hi[a], hi[a]) : hi[a];
      }
      bx.on = 1;
    }
  }
  return out;
}

// The lists of local time stepping: the tiles (of the flag-free list) that
// meet a wider box and those of the blocks that are not refined, ranges per
// kind; the gather workgroups whose own face nodes meet a wider box.  The
// scratch state is cleared when the lists are rebuilt (it must be zero off
// the tiles of the operator).
sbp_status lts_lists(sbp_ctx* c) {
  const int threads = c->tx * c->ty;
  std::vector<Tile> nt, ft;
  for (int kind : kKindOrder.k) {
    c->nk_t0[kind] = (int)nt.size();
    c->fk_t0x[kind] = (int)ft.size();
    for (int t = c->kind_t0[kind]; t < c->kind_t1[kind]; ++t) {
      const Tile& tl = c->bare[t];
      if (!c->lts_tbox[tl.block].refined) ft.push_back(tl);
      const LtsBox& bx = c->lts_tbox[tl.block];
      if (!bx.on) continue;
      const HostBlock& b = c->blocks[tl.block];
      const long long sx = b.n[0] + 2, plane = sx * (b.n[1] + 2);
      bool hit = false;
      for (int k = tl.z0; k < tl.z0 + c->cz && !hit; ++k) {
        if (k < bx.lo[2] || k > bx.hi[2]) continue;
        for (long long q = tl.q0; q < std::min<long long>(tl.q0 + threads, plane) && !hit; ++q) {
          const int j = (int)(q / sx), i = (int)(q - j * sx);
          hit = i >= bx.lo[0] && i <= bx.hi[0] && j >= bx.lo[1] && j <= bx.hi[1];
        }
      }
      if (hit) nt.push_back(tl);
    }
    c->nk_t1[kind] = (int)nt.size();
    c->fk_t1x[kind] = (int)ft.size();
  }
  // gather workgroups: own face nodes (r0, r1) along the job's tangential
  // axes, the face at node 0 or at the far end of its normal axis
  std::vector<GatherWG> gw[2], fw[2];
  for (int g = 0; g < 2; ++g)
    for (const GatherWG& w : c->hwg[g]) {
      const FaceJob& J = c->hjobs[g][w.job];
      // the ordinary step needs no face of or from a refined block: those
      // values reach only E nodes of the near boxes, which the recursion
      // replaces
      if (!c->lts_tbox[J.block].refined && !c->lts_tbox[J.nb].refined) fw[g].push_back(w);
      const LtsBox& bx = c->lts_tbox[J.block];
      if (!bx.on) continue;
      const int ax = J.face >> 1, n = c->blocks[J.block].n[ax];
      if ((J.face & 1) ? bx.hi[ax] < n : bx.lo[ax] > 0) continue;
      const long long tot = (long long)J.ext[0] * J.ext[1];
      bool hit = false;
      for (long long id = w.first; id < std::min<long long>(w.first + 256, tot) && !hit; ++id) {
        const int r0 = (int)(id % J.ext[0]), r1 = (int)(id / J.ext[0]);
        hit = r0 >= bx.lo[J.t_axis[0]] && r0 <= bx.hi[J.t_axis[0]] && r1 >= bx.lo[J.t_axis[1]] &&
              r1 <= bx.hi[J.t_axis[1]];
      }
      if (hit) gw[g].push_back(w);
    }
  auto upload = [&](auto& dst, size_t& cap, const auto& src) -> bool {
    using E = typename std::decay<decltype(src)>::type::value_type;
    if (src.size() > cap || !dst) {
      dfree(c, dst);
      dst = (std::remove_reference_t<decltype(dst)>)dalloc(c, std::max<size_t>(src.size(), 1) * sizeof(E));
      if (!dst) return false;
      cap = std::max<size_t>(src.size(), 1);
    }
    return src.empty() || hipMemcpyAsync(dst, src.data(), src.size() * sizeof(E), hipMemcpyHostToDevice,
                                         c->stream) == hipSuccess;
  };
  size_t gcap[4] = {0, 0, 0, 0};
  for (int g = 0; g < 2; ++g) {
    dfree(c, c->d_nwg[g]);
    dfree(c, c->d_fwg[g]);
    c->d_nwg[g] = c->d_fwg[g] = nullptr;
  }
  if (!upload(c->d_near, c->near_cap, nt) || !upload(c->d_far, c->far_cap, ft) ||
      !upload(c->d_nwg[0], gcap[0], gw[0]) || !upload(c->d_nwg[1], gcap[1], gw[1]) ||
      !upload(c->d_fwg[0], gcap[2], fw[0]) || !upload(c->d_fwg[1], gcap[3], fw[1]))
    return fail(c, SBP_ENOMEM, "local time stepping list allocation failed");
  // energy partial sums: one per tile of the whole list
  dfree(c, c->lts_part);
  c->lts_part = (double*)dalloc(c, std::max<size_t>(c->bare.size(), 1) * sizeof(double));
  if (!c->lts_part) return fail(c, SBP_ENOMEM, "local time stepping list allocation failed");
  c->nnear = (int)nt.size();
  c->nfar = (int)ft.size();
  for (int g = 0; g < 2; ++g) {
    c->nnwg[g] = (int)gw[g].size();
    c->nfwg[g] = (int)fw[g].size();
  }
  if (c->near_built) HIPCHK(c, hipMemsetAsync(c->lts_s, 0, c->pool_elems * elem_size(c), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));  // the host lists are locals
  c->near_dirty = false;
  c->near_built = true;
  return SBP_OK;
}

// ------------------------------------------------ allocation-free stepping
// Scratch memory of sbp_step_static: the energy partial sums of a step
// (kStaticPartials doubles) followed by the interface face buffers.  One
// copy per GPU, held until the process ends.  In host code `scratch` is a
// host-side stand-in: its address on each device comes from
// hipGetSymbolAddress (static_scratch), and only that address is handed to
// kernels.
constexpr size_t kStaticBytes = size_t(16) << 20;
constexpr size_t kStaticDoubles = kStaticBytes / sizeof(double);
constexpr size_t kStaticPartials = size_t(1) << 18;
static __device__ __align__(256) double scratch[kStaticDoubles];

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;  // device -> address of `scratch` there

// Zeroes n doubles (a kernel rather than a memset, so that a caller may
// capture the call in a graph).
__global__ __launch_bounds__(256) void k_zero(double* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Address of `scratch` on `device`, which must be current: looked up once
// per device and kept.
hipError_t static_scratch(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = g_scratch_ptr.emplace(device, (double*)p).first;
  }
  *out = it->second;
  return hipSuccess;
}

}  // namespace

// ===================================================================== ABI
extern "C" {

sbp_status sbp_create(sbp_ctx** out, sbp_prec prec, void* hip_stream, sbp_alloc_fn alloc,
                      sbp_free_fn free_fn, void* user) {
  if (!out) return SBP_EINVAL;
  *out = nullptr;
  if (prec != SBP_FP64 && prec != SBP_FP32) return SBP_EINVAL;
  if ((alloc == nullptr) != (free_fn == nullptr)) return SBP_EINVAL;
  sbp_ctx* c = new (std::nothrow) sbp_ctx();
  if (!c) return SBP_ENOMEM;
  c->prec = prec;
  c->stream = (hipStream_t)hip_stream;
  c->alloc = alloc;
  c->free_fn = free_fn;
  c->user = user;
  if (hipGetDevice(&c->device) != hipSuccess || static_scratch(c->device, &c->scratch) != hipSuccess) {
    delete c;
    return SBP_EHIP;
  }
  *out = c;
  return SBP_OK;
}

sbp_status sbp_add_block(sbp_ctx* c, int nx, int ny, int nz, double dx, double dy, double dz,
                         double x0, double y0, double z0, const double* eps_r, const double* mu_r,
                         const double* sigma, int* block_id) {
  if (!c) return SBP_EINVAL;
  if (c->finalized) return fail(c, SBP_ESTATE, "add_block after finalize");
  if (nx < 4 || ny < 4 || nz < 4)
    return fail(c, SBP_EINVAL, "a block needs at least 4 cells per axis (Appendix closures)");
  if (!(dx > 0 && dy > 0 && dz > 0)) return fail(c, SBP_EINVAL, "cell sizes must be positive");
  {
    // each component array (node box, planes padded to 64 nodes) below 4 GiB:
    // the step kernels address it with 32-bit byte offsets
    const long long sxy = ((long long)(nx + 2) * (ny + 2) + 63) / 64 * 64;
    const long long bytes = sxy * (nz + 2) * (c->prec == SBP_FP64 ? 8 : 4);
    if (bytes >= (1LL << 32) - (1LL << 20))
      return fail(c, SBP_EINVAL, "a block's component array (node box (nx+2)(ny+2)(nz+2)) must stay below 4 GiB");
  }
  HostBlock b;
  b.n[0] = nx; b.n[1] = ny; b.n[2] = nz;
  b.h[0] = dx; b.h[1] = dy; b.h[2] = dz;
  b.x0[0] = x0; b.x0[1] = y0; b.x0[2] = z0;
  const size_t nc = (size_t)nx * ny * nz;
  for (int f = 0; f < 6; ++f) {
    b.faces[f] = SBP_PEC;
    b.iface[f] = -1;
  }
  auto take = [&](const double* p, std::vector<double>& v, bool positive) -> bool {
    if (!p) return true;
    v.assign(p, p + nc);
    for (double x : v)
      if (!std::isfinite(x) || (positive ? !(x > 0) : x < 0)) return false;
    return true;
  };
  if (!take(eps_r, b.eps, true) || !take(mu_r, b.mu, true) || !take(sigma, b.sig, false))
    return fail(c, SBP_EINVAL, "materials must be finite; eps_r, mu_r > 0, sigma >= 0");
  c->blocks.push_back(std::move(b));
  if (block_id) *block_id = (int)c->blocks.size() - 1;
  return SBP_OK;
}

sbp_status sbp_set_face_bc(sbp_ctx* c, int block, int face, sbp_bc bc) {
  if (!c) return SBP_EINVAL;
  if (c->finalized) return fail(c, SBP_ESTATE, "set_face_bc after finalize");
  if (!check_block(c, block) || face < 0 || face > 5) return fail(c, SBP_EINVAL, "bad block or face");
  if (bc != SBP_PEC && bc != SBP_PMC && bc != SBP_ABC1 && bc != SBP_CPML) return fail(c, SBP_EINVAL, "bad face treatment");
  c->blocks[block].faces[face] = bc;
  return SBP_OK;
}

sbp_status sbp_connect(sbp_ctx* c, int a, int fa, int b, int fb, int ratio) {
  if (!c) return SBP_EINVAL;
  if (c->finalized) return fail(c, SBP_ESTATE, "connect after finalize");
  if (!check_block(c, a) || !check_block(c, b) || a == b) return fail(c, SBP_EINVAL, "bad blocks");
  if (fa < 0 || fa > 5 || fb < 0 || fb > 5) return fail(c, SBP_EINVAL, "bad face");
  if (fa / 2 != fb / 2 || fa % 2 == fb % 2) return fail(c, SBP_EINVAL, "faces must be opposite faces of one axis");
  if (ratio != 1 && ratio != 2) return fail(c, SBP_EINVAL, "ratio must be 1 or 2");
  HostBlock &A = c->blocks[a], &B = c->blocks[b];
  if (A.iface[fa] >= 0 || B.iface[fb] >= 0) return fail(c, SBP_EINVAL, "face already coupled");
  if (A.part_of >= 0 || B.part_of >= 0) return fail(c, SBP_EINVAL, "a complex block cannot also have interfaces");
  const int ax = fa / 2;
  const double tol = 1e-9;
  auto close = [&](double u, double v, double scale) { return std::fabs(u - v) <= tol * scale; };
  const double la = A.n[ax] * A.h[ax], lb = B.n[ax] * B.h[ax];
  const double pa = A.x0[ax] + (fa % 2 ? la : 0.0), pb = B.x0[ax] + (fb % 2 ? lb : 0.0);
  if (!close(pa, pb, std::max(la, lb))) return fail(c, SBP_EINVAL, "interface faces are not coincident");
  for (int t = 0; t < 3; ++t) {
    if (t == ax) continue;
    if (B.n[t] != ratio * A.n[t]) return fail(c, SBP_EINVAL, "interface face extents do not match the ratio");
    const double lt = A.n[t] * A.h[t];
    if (!close(A.x0[t], B.x0[t], lt) || !close(lt, B.n[t] * B.h[t], lt))
      return fail(c, SBP_EINVAL, "interface faces do not cover each other");
    if (ratio == 2 && A.n[t] < 6) return fail(c, SBP_EINVAL, "1:2 interfaces need >= 6 coarse cells along the face");
  }
  c->ifaces.push_back(HostIface{a, fa, b, fb, ratio});
  A.iface[fa] = (int)c->ifaces.size() - 1;
  B.iface[fb] = (int)c->ifaces.size() - 1;
  return SBP_OK;
}

sbp_status sbp_set_periodic(sbp_ctx* c, int block, int block_im, int axis, double alpha) {
  if (!c) return SBP_EINVAL;
  if (c->finalized) return fail(c, SBP_ESTATE, "set_periodic after finalize");
  if (!check_block(c, block)) return fail(c, SBP_EINVAL, "bad block");
  if (axis < 0 || axis > 2) return fail(c, SBP_EINVAL, "bad axis");
  if (!std::isfinite(alpha)) return fail(c, SBP_EINVAL, "phase must be finite");
  const int lo = 2 * axis, hi = 2 * axis + 1;
  HostBlock& R = c->blocks[block];
  if (R.iface[lo] >= 0 || R.iface[hi] >= 0) return fail(c, SBP_EINVAL, "face already coupled");
  if (block_im < 0) {
    if (alpha != 0.0) return fail(c, SBP_EINVAL, "a Bloch phase needs the block of the imaginary part");
    if (R.part_of >= 0) return fail(c, SBP_EINVAL, "the block holds part of a complex field: name the imaginary part");
  } else {
    if (!check_block(c, block_im) || block_im == block) return fail(c, SBP_EINVAL, "bad imaginary-part block");
    const HostBlock& I = c->blocks[block_im];
    for (int t = 0; t < 3; ++t)
      if (I.n[t] != R.n[t] || I.h[t] != R.h[t])
        return fail(c, SBP_EINVAL, "the two parts of a complex block must have the same cells and spacings");
    if (I.iface[lo] >= 0 || I.iface[hi] >= 0) return fail(c, SBP_EINVAL, "face already coupled");
    if ((R.part_of >= 0 && (R.part_of != block_im || R.imag)) || (I.part_of >= 0 && (I.part_of != block || !I.imag)))
      return fail(c, SBP_EINVAL, "a complex block keeps one imaginary-part block on every periodic axis");
    // the other faces of the two parts must not couple them to other blocks
    for (int f = 0; f < 6; ++f)
      if ((R.iface[f] >= 0 && c->ifaces[R.iface[f]].a != c->ifaces[R.iface[f]].b) ||
          (I.iface[f] >= 0 && c->ifaces[I.iface[f]].a != c->ifaces[I.iface[f]].b))
        return fail(c, SBP_EINVAL, "a complex block cannot also have interfaces");
  }
  auto add = [&](int b, int partner, int im) {
    HostIface f{b, hi, b, lo, 1};
    f.partner = partner;
    f.im = im;
    f.alpha = alpha;
    c->ifaces.push_back(f);
    c->blocks[b].iface[lo] = c->blocks[b].iface[hi] = (int)c->ifaces.size() - 1;
  };
  add(block, block_im, 0);
  if (block_im >= 0) {
    add(block_im, block, 1);
    c->blocks[block].part_of = block_im;
    c->blocks[block_im].part_of = block;
    c->blocks[block_im].imag = 1;
  }
  return SBP_OK;
}

sbp_status sbp_set_tfsf(sbp_ctx* c, int block, const int box[6], int axis, sbp_comp pol, int margin, int src_cell,
                        sbp_wave w, const double p[3], double amplitude) {
  if (!c) return SBP_EINVAL;
  if (c->finalized) return fail(c, SBP_ESTATE, "set_tfsf after finalize");
  if (c->tf_on) return fail(c, SBP_ESTATE, "one TF/SF box per context");
  if (!check_block(c, block) || !box) return fail(c, SBP_EINVAL, "bad block");
  if (axis < 0 || axis > 2) return fail(c, SBP_EINVAL, "bad axis");
  if (pol < SBP_EX || pol > SBP_EZ || (int)pol == axis) return fail(c, SBP_EINVAL, "the polarisation is an E component across the axis");
  HostBlock& b = c->blocks[block];
  for (int a = 0; a < 3; ++a)
    if (box[2 * a] < 4 || box[2 * a + 1] > b.n[a] - 4 || box[2 * a] >= box[2 * a + 1])
      return fail(c, SBP_EINVAL, "the TF/SF box must lie at least 4 cells inside the block");
  if (margin < 1 || margin > (1 << 20)) return fail(c, SBP_EINVAL, "margin must be in 1 .. 2^20");
  const int L = b.n[axis] + 2 * margin;
  if (src_cell + margin < 1 || src_cell + margin > L - 1) return fail(c, SBP_EINVAL, "source cell outside the line");
  if (w != SBP_GAUSS && w != SBP_MODGAUSS) return fail(c, SBP_EINVAL, "bad waveform");
  if (!p || !(p[0] > 0)) return fail(c, SBP_EINVAL, "source width must be positive");
  c->tf_on = true;
  c->tf_block = block;
  for (int f = 0; f < 6; ++f) c->tf_box[f] = box[f];
  c->tf_axis = axis;
  c->tf_pol = pol;
  c->tf_margin = margin;
  c->tf_cell = src_cell;
  std::memset(&c->tf_srcdef, 0, sizeof(Source));
  c->tf_srcdef.comp = pol;
  c->tf_srcdef.i = c->tf_srcdef.j = c->tf_srcdef.k = -1;  // on no block node
  c->tf_srcdef.wave = w;
  c->tf_srcdef.tw = p[0];
  c->tf_srcdef.t0 = p[1];
  c->tf_srcdef.f0 = p[2];
  c->tf_srcdef.amp = amplitude;
  b.tfsf = 1;
  return SBP_OK;
}

sbp_status sbp_add_source(sbp_ctx* c, int block, sbp_comp comp, int i, int j, int k, sbp_wave w,
                          const double p[3], double amplitude, int* id) {
  if (!c) return SBP_EINVAL;
  if (c->finalized) return fail(c, SBP_ESTATE, "add_source after finalize");
  if (!check_block(c, block) || comp < SBP_EX || comp > SBP_EZ) return fail(c, SBP_EINVAL, "sources act on E components");
  const HostBlock& b = c->blocks[block];
  if (i < 0 || j < 0 || k < 0 || i >= comp_dim(b, comp, 0) || j >= comp_dim(b, comp, 1) || k >= comp_dim(b, comp, 2))
    return fail(c, SBP_EINVAL, "source node outside the component grid");
  if (w != SBP_GAUSS && w != SBP_MODGAUSS) return fail(c, SBP_EINVAL, "bad waveform");
  if (!p || !(p[0] > 0)) return fail(c, SBP_EINVAL, "source width must be positive");
  HostSource s;
  s.block = block;
  std::memset(&s.s, 0, sizeof(s.s));
  s.s.comp = comp; s.s.i = i; s.s.j = j; s.s.k = k;
  s.s.wave = w;
  s.s.tw = p[0]; s.s.t0 = p[1]; s.s.f0 = p[2];
  s.s.amp = amplitude;
  c->srcs.push_back(s);
  if (id) *id = (int)c->srcs.size() - 1;
  return SBP_OK;
}

sbp_status sbp_add_probe(sbp_ctx* c, int block, sbp_comp comp, int i, int j, int k, int* id) {
  if (!c) return SBP_EINVAL;
  if (c->finalized) return fail(c, SBP_ESTATE, "add_probe after finalize");
  if (!check_block(c, block) || comp < SBP_EX || comp > SBP_HZ) return fail(c, SBP_EINVAL, "bad block or component");
  const HostBlock& b = c->blocks[block];
  if (i < 0 || j < 0 || k < 0 || i >= comp_dim(b, comp, 0) || j >= comp_dim(b, comp, 1) || k >= comp_dim(b, comp, 2))
    return fail(c, SBP_EINVAL, "probe node outside the component grid");
  HostProbe p;
  p.block = block;
  p.p.comp = comp; p.p.i = i; p.p.j = j; p.p.k = k;
  c->prbs.push_back(p);
  if (id) *id = (int)c->prbs.size() - 1;
  return SBP_OK;
}

sbp_status sbp_finalize(sbp_ctx* c, double cfl, int force, long history, double* dt_out) {
  if (!c) return SBP_EINVAL;
  if (c->finalized) return fail(c, SBP_ESTATE, "already finalized");
  if (c->blocks.empty()) return fail(c, SBP_ESTATE, "no blocks");
  if (!(cfl > 0)) return fail(c, SBP_EINVAL, "cfl_fraction must be positive");
  if (cfl > 1.0 && !force) return fail(c, SBP_EUNSTABLE, "cfl_fraction above the stability limit");
  if (history < 2) history = 2;
  if (history > (1L << 26)) return fail(c, SBP_EINVAL, "history too long");
  HIPCHK(c, hipSetDevice(c->device));
  // time step: Yee limit of the finest block
  double lim = 1e300;
  for (auto& b : c->blocks)
    lim = std::min(lim, 1.0 / (kC0 * std::sqrt(1.0 / (b.h[0] * b.h[0]) + 1.0 / (b.h[1] * b.h[1]) + 1.0 / (b.h[2] * b.h[2]))));
  c->dt = cfl * lim;
  c->history = history;
  // per-source / per-probe: group by block
  std::vector<Source> dsrc;
  std::vector<Probe> dprb;
  c->hblocks.assign(c->blocks.size(), DevBlock());
  c->probe_order.assign(c->prbs.size(), 0);
  size_t foff = 0, coff = 0, fboff = 0, psi = 0;
  std::vector<double> pml;
  for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
    HostBlock& b = c->blocks[bi];
    DevBlock& d = c->hblocks[bi];
    std::memset(&d, 0, sizeof(d));
    for (int a = 0; a < 3; ++a) {
      d.n[a] = b.n[a];
      d.h[a] = b.h[a];
      d.ih[a] = 1.0 / b.h[a];
    }
    d.sx = b.n[0] + 2;
    // planes padded to 64 nodes: every wave's centre accesses start on a 256 B
    // (fp32) boundary when the tiles start on 64-node boundaries
    d.sxy = (d.sx * (b.n[1] + 2) + 63) / 64 * 64;
    d.csz = d.sxy * (b.n[2] + 2);
    d.foff = (long long)foff;
    foff += 6 * (size_t)d.csz;
    d.coff = (long long)coff;
    coff += (size_t)b.n[0] * b.n[1] * b.n[2];
    d.eps_r0 = 1.0;
    d.mu_r0 = 1.0;
    d.sig0 = 0.0;
    d.abc_mask = 0;
    d.iface_mask = 0;
    for (int f = 0; f < 6; ++f) {
      if (b.iface[f] >= 0) {
        d.iface_mask |= 1 << f;
        const int ax = f / 2;
        const int e0 = ax == 0 ? b.n[1] + 2 : b.n[0] + 2;
        const int e1 = ax == 2 ? b.n[1] + 2 : b.n[2] + 2;
        d.fsz[f] = (long long)e0 * e1;
        d.fboff[f] = (long long)fboff;
        fboff += 4 * (size_t)d.fsz[f];
      } else {
        d.fsz[f] = 0;
        d.fboff[f] = 0;
        if (b.faces[f] == SBP_ABC1) d.abc_mask |= 1 << f;
      }
    }
    build_rows(b, d);
    if (has_pml(b)) {  // twelve psi arrays (six H, six E terms) over the node box
      d.pml_stride = std::max(b.n[0], std::max(b.n[1], b.n[2])) + 2;
      d.pml_off = (long long)pml.size();
      pml_profiles(c, b, d.pml_stride, pml);
      d.psi_off = (long long)psi;
      psi += 12 * (size_t)d.csz;
    }
    d.db_u = c->dt / (kMu0 * d.mu_r0);
    d.cb_u = c->dt / (kEps0 * d.eps_r0);
    d.dte0x4 = 4.0 * c->dt / kEps0;
    d.hdte0 = c->dt / (2.0 * kEps0);
    d.dtm0x2 = 2.0 * c->dt / kMu0;
    d.ke = 0.5 * kEps0 * b.h[0] * b.h[1] * b.h[2];
    d.kh = 0.5 * kMu0 * b.h[0] * b.h[1] * b.h[2];

    d.src0 = (int)dsrc.size();
    for (auto& s : c->srcs)
      if (s.block == (int)bi) dsrc.push_back(s.s);
    d.nsrc = (int)dsrc.size() - d.src0;
    d.prb0 = (int)dprb.size();
    for (size_t p = 0; p < c->prbs.size(); ++p)
      if (c->prbs[p].block == (int)bi) {
        c->probe_order[p] = (int)dprb.size();
        dprb.push_back(c->prbs[p].p);
      }
    d.nprb = (int)dprb.size() - d.prb0;
  }
  // the kernels track at most two sources and two E (two H) probes per
  // (block, i, j) node column
  for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
    const DevBlock& d = c->hblocks[bi];
    for (int q = 0; q < d.nsrc; ++q) {
      int cnt = 0;
      for (int r = 0; r < d.nsrc; ++r)
        cnt += dsrc[d.src0 + r].i == dsrc[d.src0 + q].i && dsrc[d.src0 + r].j == dsrc[d.src0 + q].j;
      if (cnt > 2) return fail(c, SBP_EINVAL, "more than two sources on one node column");
    }
    for (int q = 0; q < d.nprb; ++q) {
      int cnt = 0;
      const Probe& P = dprb[d.prb0 + q];
      for (int r = 0; r < d.nprb; ++r) {
        const Probe& R = dprb[d.prb0 + r];
        cnt += R.i == P.i && R.j == P.j && (R.comp >= 3) == (P.comp >= 3);
      }
      if (cnt > 2) return fail(c, SBP_EINVAL, "more than two probes of one field on one node column");
    }
  }
  if (c->tf_on) {  // the incident source follows the point sources of every block
    const HostBlock& b = c->blocks[c->tf_block];
    for (int f = 0; f < 6; ++f)
      if (b.iface[f] >= 0) return fail(c, SBP_EINVAL, "the TF/SF block takes no interface or periodic faces");
    for (int f = 0; f < 6; ++f) {
      const int a = f / 2;
      const int gap = (f & 1) ? b.n[a] - c->tf_box[f] : c->tf_box[f];
      if (b.iface[f] < 0 && b.faces[f] == SBP_CPML && gap < c->pml_cells + 4)
        return fail(c, SBP_EINVAL, "the TF/SF box must lie at least 4 cells inside the absorbing layers");
    }
    c->tf_sidx = (int)dsrc.size();
    dsrc.push_back(c->tf_srcdef);
    c->tf_len = b.n[c->tf_axis] + 2 * c->tf_margin;
  }
  c->pool_elems = foff;
  c->ncells = coff;
  c->pool = dalloc(c, foff * elem_size(c));
  c->pool2 = c->fused ? dalloc(c, foff * elem_size(c)) : c->pool;
  c->d_blocks = (DevBlock*)dalloc(c, c->hblocks.size() * sizeof(DevBlock));
  c->d_src = (Source*)dalloc(c, std::max<size_t>(dsrc.size(), 1) * sizeof(Source));
  c->d_srcval = (double*)dalloc(c, std::max<size_t>(dsrc.size(), 1) * sizeof(double));
  c->nsrc_total = (int)dsrc.size();
  c->d_prb = (Probe*)dalloc(c, std::max<size_t>(dprb.size(), 1) * sizeof(Probe));
  c->d_energy = (double*)dalloc(c, (size_t)history * sizeof(double));
  c->d_probes = (double*)dalloc(c, std::max<size_t>(dprb.size(), 1) * (size_t)history * sizeof(double));
  c->d_st = (StepState*)dalloc(c, sizeof(StepState));
  c->d_face = (double*)dalloc(c, std::max<size_t>(fboff, 1) * sizeof(double));
  c->face_elems = std::max<size_t>(fboff, 1);
  c->psi_elems = psi;
  if (c->tf_on) {
    c->d_line = (double*)dalloc(c, line_bytes(c));
    c->d_tf = (TfDesc*)dalloc(c, sizeof(TfDesc));
    if (!c->d_line || !c->d_tf) return fail(c, SBP_ENOMEM, "device allocation failed");
    HIPCHK(c, hipMemsetAsync(c->d_line, 0, line_bytes(c), c->stream));
    const HostBlock& b = c->blocks[c->tf_block];
    const int pr = c->tf_axis, ep = c->tf_pol, hq = 3 - pr - ep;
    // signs of d_axis in the H equation of H_hq and the E equation of E_ep
    // (curl part of H_c: +d_{c+2} E_{c+1} - d_{c+1} E_{c+2}; the same for E)
    const double sh = (hq + 2) % 3 == pr ? 1.0 : -1.0, se = (ep + 1) % 3 == pr ? 1.0 : -1.0;
    TfDesc t;
    t.e1 = c->d_line;
    t.h1 = c->d_line + c->tf_len + 1;
    t.ch = c->dt * sh / (kMu0 * b.h[pr]);
    t.ce = c->dt * se / (kEps0 * b.h[pr]);
    t.block = c->tf_block;
    t.axis = pr;
    t.ep = ep;
    t.hq = hq;
    t.margin = c->tf_margin;
    t.len = c->tf_len;
    t.src = c->tf_cell + c->tf_margin;
    t.sidx = c->tf_sidx;
    for (int a = 0; a < 3; ++a) {
      t.lo[a] = c->tf_box[2 * a];
      t.hi[a] = c->tf_box[2 * a + 1];
    }
    // the curl terms that difference E_ep (in the H components other than
    // ep) and H_hq (in the E components other than hq): with the curl parts
    // H_c: +d_{c+2} E_{c+1} - d_{c+1} E_{c+2} and E_c: +d_{c+1} H_{c+2} -
    // d_{c+2} H_{c+1}, the term's axis is the one left over, its sign + when
    // it is the first term
    for (int m = 0, cc = 0; cc < 3; ++cc) {
      if (cc == ep) continue;
      const bool first = (cc + 1) % 3 == ep;
      t.h_comp[m] = cc;
      t.h_ax[m] = first ? (cc + 2) % 3 : (cc + 1) % 3;
      t.h_sg[m++] = first ? 1.0 : -1.0;
    }
    for (int m = 0, cc = 0; cc < 3; ++cc) {
      if (cc == hq) continue;
      const bool first = (cc + 2) % 3 == hq;
      t.e_comp[m] = cc;
      t.e_ax[m] = first ? (cc + 1) % 3 : (cc + 2) % 3;
      t.e_sg[m++] = first ? 1.0 : -1.0;
    }
    HIPCHK(c, hipMemcpy(c->d_tf, &t, sizeof(t), hipMemcpyHostToDevice));
  }
  c->d_pml = dalloc(c, std::max<size_t>(pml.size(), 1) * elem_size(c));
  c->d_psi = dalloc(c, std::max<size_t>(psi, 1) * elem_size(c));
  if (!c->d_pml || !c->d_psi) return fail(c, SBP_ENOMEM, "device allocation failed");
  if (!pml.empty()) {
    if (c->prec == SBP_FP64) {
      HIPCHK(c, hipMemcpy(c->d_pml, pml.data(), pml.size() * 8, hipMemcpyHostToDevice));
    } else {
      std::vector<float> f(pml.begin(), pml.end());
      HIPCHK(c, hipMemcpy(c->d_pml, f.data(), f.size() * 4, hipMemcpyHostToDevice));
    }
  }
  HIPCHK(c, hipMemsetAsync(c->d_psi, 0, std::max<size_t>(psi, 1) * elem_size(c), c->stream));
  if (!c->pool || !c->pool2 || !c->d_blocks || !c->d_src || !c->d_srcval || !c->d_prb || !c->d_energy || !c->d_probes || !c->d_st || !c->d_face)
    return fail(c, SBP_ENOMEM, "device allocation failed");
  HIPCHK(c, hipMemsetAsync(c->pool, 0, foff * elem_size(c), c->stream));
  if (c->pool2 != c->pool) HIPCHK(c, hipMemsetAsync(c->pool2, 0, foff * elem_size(c), c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_energy, 0, (size_t)history * sizeof(double), c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_probes, 0, std::max<size_t>(dprb.size(), 1) * (size_t)history * sizeof(double), c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_st, 0, sizeof(StepState), c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_srcval, 0, std::max<size_t>(dsrc.size(), 1) * sizeof(double), c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_face, 0, std::max<size_t>(fboff, 1) * sizeof(double), c->stream));
  if (!dsrc.empty())
    HIPCHK(c, hipMemcpyAsync(c->d_src, dsrc.data(), dsrc.size() * sizeof(Source), hipMemcpyHostToDevice, c->stream));
  if (!dprb.empty())
    HIPCHK(c, hipMemcpyAsync(c->d_prb, dprb.data(), dprb.size() * sizeof(Probe), hipMemcpyHostToDevice, c->stream));
  // interface gather jobs
  std::vector<FaceJob> je, jh;
  std::vector<Taps> taps;
  for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
    const HostBlock& b = c->blocks[bi];
    for (int f = 0; f < 6; ++f) {
      if (b.iface[f] < 0) continue;
      const HostIface& I = c->ifaces[b.iface[f]];
      const bool is_a = I.a == (int)bi && I.fa == f;
      const int nb = is_a ? I.b : I.a;
      const int fn = is_a ? I.fb : I.fa;
      const int role = I.ratio == 1 ? 0 : (is_a ? 2 : 1);  // 2: own coarse, 1: own fine
      const int ax = f / 2;
      const int ta[2] = {ax == 0 ? 1 : 0, ax == 2 ? 1 : 2};
      for (int is_h = 0; is_h < 2; ++is_h)
        for (int slot = 0; slot < 2; ++slot) {
          FaceJob J;
          std::memset(&J, 0, sizeof(J));
          J.block = (int)bi;
          J.face = f;
          J.is_h = is_h;
          J.slot = slot;
          J.comp = is_h ? 3 + ta[slot] : ta[slot];
          J.nb = nb;
          // EPBC1-EPBC6: the high face takes e^{-j alpha} times the low
          // face's values, the low face e^{+j alpha} times the high face's;
          // for fields split into real and imaginary parts the part held by
          // the other block enters with +-sin(alpha)
          J.nb2 = I.partner;
          J.w1 = I.partner >= 0 ? std::cos(I.alpha) : 1.0;
          J.w2 = I.partner >= 0 ? ((f % 2) ? 1.0 : -1.0) * (I.im ? -1.0 : 1.0) * std::sin(I.alpha) : 0.0;
          const HostBlock& N = c->blocks[nb];
          // face-normal index of the neighbour's face: "+" along the normal for
          // tangential E (0 or n), "-" for tangential H (0 or n+1)
          J.nb_idx = (fn % 2) ? (is_h ? N.n[ax] + 1 : N.n[ax]) : 0;
          for (int q = 0; q < 2; ++q) {
            J.t_axis[q] = ta[q];
            const bool plus = kPlus[J.comp][ta[q]];
            J.ext[q] = plus ? b.n[ta[q]] + 1 : b.n[ta[q]] + 2;
            J.taps_off[q] = (long long)taps.size();
            if (!axis_taps(plus, b.n[ta[q]], role, taps))
              return fail(c, SBP_EINVAL, "interface interpolation wider than the tap limit");
          }
          J.unit = role == 0 ? 1 : 0;
          (is_h ? jh : je).push_back(J);
        }
    }
  }
  c->njobs_e = (int)je.size();
  c->njobs_h = (int)jh.size();
  // each job's face nodes in runs of 256, one workgroup per run
  auto wg_table = [](const std::vector<FaceJob>& jobs) {
    std::vector<GatherWG> t;
    for (size_t q = 0; q < jobs.size(); ++q)
      for (int f = 0; f < jobs[q].ext[0] * jobs[q].ext[1]; f += 256) t.push_back(GatherWG{(int)q, f});
    return t;
  };
  const std::vector<GatherWG> we = wg_table(je), wh = wg_table(jh);
  c->nwg_e = (int)we.size();
  c->nwg_h = (int)wh.size();
  c->hjobs[0] = je;
  c->hjobs[1] = jh;
  c->hwg[0] = we;
  c->hwg[1] = wh;
  if (!je.empty()) {
    c->d_jobs_e = (FaceJob*)dalloc(c, je.size() * sizeof(FaceJob));
    c->d_jobs_h = (FaceJob*)dalloc(c, jh.size() * sizeof(FaceJob));
    c->d_wg_e = (GatherWG*)dalloc(c, we.size() * sizeof(GatherWG));
    c->d_wg_h = (GatherWG*)dalloc(c, wh.size() * sizeof(GatherWG));
    if (!c->d_wg_e || !c->d_wg_h) return fail(c, SBP_ENOMEM, "device allocation failed");
    HIPCHK(c, hipMemcpyAsync(c->d_wg_e, we.data(), we.size() * sizeof(GatherWG), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_wg_h, wh.data(), wh.size() * sizeof(GatherWG), hipMemcpyHostToDevice, c->stream));
    c->d_taps = (Taps*)dalloc(c, taps.size() * sizeof(Taps));
    if (!c->d_jobs_e || !c->d_jobs_h || !c->d_taps) return fail(c, SBP_ENOMEM, "device allocation failed");
    HIPCHK(c, hipMemcpyAsync(c->d_jobs_e, je.data(), je.size() * sizeof(FaceJob), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_jobs_h, jh.data(), jh.size() * sizeof(FaceJob), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_taps, taps.data(), taps.size() * sizeof(Taps), hipMemcpyHostToDevice, c->stream));
  }
  HIPCHK(c, hipEventCreate(&c->ev0));
  HIPCHK(c, hipEventCreate(&c->ev1));
  c->finalized = true;
  sbp_status st = upload_materials(c);
  if (st != SBP_OK) return st;
  if (!c->launch_set) {
    // small problems: few tiles of 8 planes leave CUs idle, and a thread's
    // march through its planes is a chain of load latencies; shorter tiles
    // fill the chip.  Measured (graph-replayed us per step; 1 / 2 / 4 / 8
    // planes at 128 threads): 16^3 fp64 11.5 / 13.6 / 18.2 / -, 40^3
    // 11.2 / 12.5 / 14.3 / 23.2 (84 tiles of 8 planes), 56^3 13.1 / 12.9 /
    // 15.2 / 19.7 (216), 72^3 17.5 / 15.2 / 17.2 / 22.9 (430), 80^3 20.1 /
    // 17.1 / 17.0 / 21.9 (583), 96^3 30.5 / 24.1 / 21.7 / 27 (988)
    long long tiles = 0;
    for (const HostBlock& b : c->blocks) {
      const long long sxy = (long long)(b.n[0] + 2) * (b.n[1] + 2);
      tiles += (sxy + c->tx * c->ty - 1) / (c->tx * c->ty) * ((b.n[2] + 2 + c->cz - 1) / c->cz);
    }
    if (c->cz == 8) c->cz = tiles < 160 ? 1 : (tiles < 512 ? 2 : (tiles < 2048 ? 4 : 8));
  }
  st = build_tiles(c);
  if (st != SBP_OK) return st;
  c->nstep = 0;
  if (dt_out) *dt_out = c->dt;
  return SBP_OK;
}

sbp_status sbp_set_materials(sbp_ctx* c, int block, const double* eps_r, const double* mu_r,
                             const double* sigma) {
  if (!c) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "set_materials before finalize");
  if (c->lts) return fail(c, SBP_ESTATE, "the context steps by local time stepping (sbp_lts_step)");
  if (!check_block(c, block)) return fail(c, SBP_EINVAL, "bad block");
  HostBlock& b = c->blocks[block];
  const size_t nc = (size_t)b.n[0] * b.n[1] * b.n[2];
  std::vector<double> e, m, s;
  if (eps_r) e.assign(eps_r, eps_r + nc);
  if (mu_r) m.assign(mu_r, mu_r + nc);
  if (sigma) s.assign(sigma, sigma + nc);
  for (double x : e) if (!(x > 0) || !std::isfinite(x)) return fail(c, SBP_EINVAL, "eps_r must be positive");
  for (double x : m) if (!(x > 0) || !std::isfinite(x)) return fail(c, SBP_EINVAL, "mu_r must be positive");
  for (double x : s) if (!(x >= 0) || !std::isfinite(x)) return fail(c, SBP_EINVAL, "sigma must be >= 0");
  const int kind_before = block_kind(b);
  const bool tabled_before = b.tabled;
  b.eps.swap(e);
  b.mu.swap(m);
  b.sig.swap(s);
  void* old[3] = {c->mat[0], c->mat[1], c->mat[2]};
  sbp_status st = upload_materials(c);
  if (st != SBP_OK) return st;
  // a block whose set of per-cell materials changed takes other kernels:
  // rebuild the tile lists (this also drops a captured graph)
  if (block_kind(b) != kind_before || b.tabled != tabled_before) return build_tiles(c);
  if (old[0] != c->mat[0] || old[1] != c->mat[1] || old[2] != c->mat[2]) drop_graph(c);
  return SBP_OK;
}

sbp_status sbp_set_launch(sbp_ctx* c, int tx, int ty, int cz, int workgroups) {
  if (!c) return SBP_EINVAL;
  const int t = tx * ty;
  if (tx < 1 || ty < 1 || (t != 64 && t != 128 && t != 256)) return fail(c, SBP_EINVAL, "tx*ty must be 64, 128 or 256");
  if (cz < 1 || cz > 1024 || workgroups < 0) return fail(c, SBP_EINVAL, "cz must be 1..1024, workgroups >= 0");
  c->tx = tx;
  c->ty = ty;
  c->cz = cz;
  c->wgs = workgroups;
  c->launch_set = true;
  if (c->finalized) return build_tiles(c);
  return SBP_OK;
}

sbp_status sbp_set_cpml(sbp_ctx* c, int cells, int order, double sigma_factor, double kappa_max, double alpha_max) {
  if (!c) return SBP_EINVAL;
  if (c->finalized) return fail(c, SBP_ESTATE, "set_cpml after finalize");
  if (cells < 1 || order < 1 || order > 8 || !(sigma_factor >= 0.0) || !(kappa_max >= 1.0) || !(alpha_max >= 0.0) ||
      !std::isfinite(sigma_factor) || !std::isfinite(kappa_max) || !std::isfinite(alpha_max))
    return fail(c, SBP_EINVAL, "CPML: cells >= 1, 1 <= order <= 8, sigma_factor >= 0, kappa_max >= 1, alpha_max >= 0");
  c->pml_cells = cells;
  c->pml_m = order;
  c->pml_sigma_factor = sigma_factor;
  c->pml_kappa_max = kappa_max;
  c->pml_alpha_max = alpha_max;
  return SBP_OK;
}

sbp_status sbp_set_cell_tables(sbp_ctx* c, int enable) {
  if (!c) return SBP_EINVAL;
  if (c->lts) return fail(c, SBP_ESTATE, "the context steps by local time stepping (sbp_lts_step)");
  c->tables_off = enable == 0;
  if (!c->finalized) return SBP_OK;
  HIPCHK(c, hipSetDevice(c->device));
  const sbp_status st = upload_materials(c);
  if (st != SBP_OK) return st;
  return build_tiles(c);  // blocks may change kind; this also drops a captured graph
}

sbp_status sbp_set_fused(sbp_ctx* c, int enable, int planes) {
  if (!c) return SBP_EINVAL;
  if (c->lts) return fail(c, SBP_ESTATE, "the context steps by local time stepping (sbp_lts_step)");
  if (planes < 4 || planes > 4096) return fail(c, SBP_EINVAL, "planes per one-pass tile must be 4..4096");
  c->fz = planes;
  drop_graph(c);
  if (c->finalized) {
    const size_t pb = c->pool_elems * elem_size(c);
    HIPCHK(c, hipSetDevice(c->device));
    if (enable && c->pool2 == c->pool) {  // second pool, holding the state too
      void* p2 = dalloc(c, pb);
      if (!p2) return fail(c, SBP_ENOMEM, "second field pool allocation failed");
      HIPCHK(c, hipMemcpyAsync(p2, c->pool, pb, hipMemcpyDeviceToDevice, c->stream));
      c->pool2 = p2;
    } else if (!enable && c->pool2 != c->pool) {  // back to one pool
      if (c->nstep & 1) HIPCHK(c, hipMemcpyAsync(c->pool, c->pool2, pb, hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      dfree(c, c->pool2);
      c->pool2 = c->pool;
    }
  }
  c->fused = enable ? 1 : 0;
  if (c->finalized) return build_tiles(c);
  return SBP_OK;
}

sbp_status sbp_get_launch(const sbp_ctx* c, int out[4]) {
  if (!c || !out) return SBP_EINVAL;
  out[0] = c->tx; out[1] = c->ty; out[2] = c->cz; out[3] = c->wgs;
  return SBP_OK;
}

sbp_status sbp_step(sbp_ctx* c, long nsteps) {
  if (!c) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "step before finalize");
  if (c->lts) return fail(c, SBP_ESTATE, "the context steps by local time stepping (sbp_lts_step)");
  if (nsteps < 0) return fail(c, SBP_EINVAL, "negative step count");
  if (nsteps == 0) return SBP_OK;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  HIPCHK(c, launch_sources(kargs(c), c->stream));  // source values of the current step
  long done = 0;
  if (c->graph_steps > 0 && nsteps >= c->graph_steps && !c->profile) {
    if (!c->gexec) {
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      sbp_status st = SBP_OK;
      for (int s = 0; s < c->graph_steps && st == SBP_OK; ++s) st = enqueue_step(c, false);
      hipGraph_t g = nullptr;
      hipError_t ee = hipStreamEndCapture(c->stream, &g);
      if (st != SBP_OK) return st;
      HIPCHK(c, ee);
      c->graph = g;
      HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    }
    while (nsteps - done >= c->graph_steps) {
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
      done += c->graph_steps;
    }
  }
  if (c->profile) {
    const size_t need = (size_t)(nsteps - done) * 6;
    while (c->kev.size() < need) {
      hipEvent_t e;
      HIPCHK(c, hipEventCreate(&e));
      c->kev.push_back(e);
    }
    c->kev_used = 0;
  }
  for (; done < nsteps; ++done) {
    sbp_status st = enqueue_step(c, c->profile);
    if (st != SBP_OK) return st;
  }
  HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  c->timed = true;
  c->nstep += nsteps;
  return SBP_OK;
}

sbp_status sbp_step_static(sbp_ctx* c, long nsteps) {
  if (!c) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "step before finalize");
  if (c->lts) return fail(c, SBP_ESTATE, "the context steps by local time stepping (sbp_lts_step)");
  if (nsteps < 0) return fail(c, SBP_EINVAL, "negative step count");
  if (!c->scratch) return fail(c, SBP_EHIP, "no static scratch on this device");
  if (c->partials_need > kStaticPartials)
    return fail(c, SBP_EINVAL,
                "launch shape needs " + std::to_string(c->partials_need) +
                    " partial sums; the static scratch holds " + std::to_string(kStaticPartials) +
                    " (larger tiles, or sbp_step)");
  if (c->face_elems > kStaticDoubles - kStaticPartials)
    return fail(c, SBP_EINVAL,
                "interfaces need " + std::to_string(c->face_elems) + " face values; the static scratch holds " +
                    std::to_string(kStaticDoubles - kStaticPartials) + " (use sbp_step)");
  if (nsteps == 0) return SBP_OK;
  HIPCHK(c, hipSetDevice(c->device));
  KArgs a = kargs(c);
  a.partials = c->scratch;
  a.face = c->scratch + kStaticPartials;
  // the face buffers hold slots no gather writes (nodes a component does not
  // have), which the kernels read as zero: clear what the last call left
  const size_t nf = c->face_elems;
  const int zb = (int)std::min<size_t>((nf + 255) / 256, 1024);
  hipLaunchKernelGGL(k_zero, dim3(zb), dim3(256), 0, c->stream, c->scratch + kStaticPartials, nf);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, launch_sources(a, c->stream));  // source values of the current step
  for (long s = 0; s < nsteps; ++s) {
    const sbp_status st = enqueue_step_on(c, a, false);
    if (st != SBP_OK) return st;
  }
  c->timed = false;
  c->nstep += nsteps;
  return SBP_OK;
}

sbp_status sbp_lts_start(sbp_ctx* c, const int* refined, int nrefined, int substeps, double dt_coarse,
                          long energy_every) {
  if (!c) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "local time stepping before finalize");
  if (c->lts) return fail(c, SBP_ESTATE, "local time stepping already started");
  if (substeps < 1 || substeps > 64) return fail(c, SBP_EINVAL, "substeps must be 1..64");
  if (!(dt_coarse > 0.0) || !std::isfinite(dt_coarse)) return fail(c, SBP_EINVAL, "dt_coarse must be positive");
  if (energy_every < 0) return fail(c, SBP_EINVAL, "energy_every must be >= 0");
  if (nrefined < 0 || (nrefined > 0 && !refined)) return fail(c, SBP_EINVAL, "bad refined-block list");
  if (c->fused) return fail(c, SBP_EINVAL, "local time stepping takes the two-pass step (sbp_set_fused 0)");
  if (!c->srcs.empty() || c->tf_on) return fail(c, SBP_EINVAL, "local time stepping takes no sources or TF/SF box");
  if (!c->prbs.empty()) return fail(c, SBP_EINVAL, "local time stepping records no probes (read the fields instead)");
  const int nb = (int)c->blocks.size();
  std::vector<int> flag(nb, 0);
  for (int q = 0; q < nrefined; ++q) {
    if (!check_block(c, refined[q])) return fail(c, SBP_EINVAL, "bad refined block");
    flag[refined[q]] = 1;
  }
  for (const HostBlock& b : c->blocks) {
    bool lossy = false;
    for (double v : b.sig) lossy = lossy || v != 0.0;
    for (int f = 0; f < 6; ++f) {
      lossy = lossy || (b.iface[f] < 0 && (b.faces[f] == SBP_ABC1 || b.faces[f] == SBP_CPML));
      if (b.iface[f] >= 0 && c->ifaces[b.iface[f]].a == c->ifaces[b.iface[f]].b)
        return fail(c, SBP_EINVAL, "local time stepping takes no periodic faces");
    }
    if (lossy) return fail(c, SBP_EINVAL, "local time stepping covers lossless blocks (no conductivity, no absorbing faces)");
  }
  HIPCHK(c, hipSetDevice(c->device));
  drop_graph(c);
  const size_t pb = c->pool_elems * elem_size(c);
  const bool sub = substeps > 1 && nrefined > 0;  // the recursion differs from the leapfrog
  const bool track = energy_every > 0;
  auto take = [&](size_t bytes) { return dalloc(c, bytes); };
  c->lts_s = take(pb);
  if (sub) {
    c->lts_w = take(pb);
    c->lts_qa = take(pb);
    c->lts_qb = take(pb);
    c->lts_ep = take(pb);
  }
  if (track) {
    c->lts_x[0] = take(pb);
    c->lts_x[1] = take(pb);
  }
  c->lts_face = (double*)take(c->face_elems * sizeof(double));
  c->lts_st = (StepState*)take(sizeof(StepState));
  c->lts_ring = (double*)take(2 * sizeof(double));
  c->lts_part = nullptr;  // sized with the tile list (lts_lists)
  c->lts_blocks = (DevBlock*)take((size_t)nb * sizeof(DevBlock));
  c->lts_cblocks = (DevBlock*)take((size_t)nb * sizeof(DevBlock));
  c->lts_boxes = (LtsBox*)take((size_t)nb * sizeof(LtsBox));
  if (!c->lts_s || (sub && (!c->lts_w || !c->lts_qa || !c->lts_qb || !c->lts_ep)) ||
      (track && (!c->lts_x[0] || !c->lts_x[1])) || !c->lts_face || !c->lts_st || !c->lts_ring ||
      !c->lts_blocks || !c->lts_cblocks || !c->lts_boxes)
    return fail(c, SBP_ENOMEM, "local time stepping buffer allocation failed");
  // descriptors with a unit time step (one step of the scratch state applies
  // B and then A: Section V's update with dt = 1) and with the coarse one
  std::vector<DevBlock> ub(c->hblocks), cb(c->hblocks);
  auto with_dt = [](DevBlock& d, double dt) {
    d.db_u = dt / (kMu0 * d.mu_r0);
    d.cb_u = dt / (kEps0 * d.eps_r0);
    d.dte0x4 = 4.0 * dt / kEps0;
    d.hdte0 = dt / (2.0 * kEps0);
    d.dtm0x2 = 2.0 * dt / kMu0;
  };
  for (size_t q = 0; q < ub.size(); ++q) {
    with_dt(ub[q], 1.0);
    with_dt(cb[q], dt_coarse);
  }
  c->lts_hbox = lts_boxes(c, flag, kLtsNear);
  c->lts_tbox = lts_boxes(c, flag, kLtsWide);
  if (!sub)
    for (LtsBox& x : c->lts_hbox) x.on = 0;
  HIPCHK(c, hipMemcpyAsync(c->lts_blocks, ub.data(), ub.size() * sizeof(DevBlock), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->lts_cblocks, cb.data(), cb.size() * sizeof(DevBlock), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->lts_boxes, c->lts_hbox.data(), nb * sizeof(LtsBox), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync(c->lts_face, 0, c->face_elems * sizeof(double), c->stream));
  HIPCHK(c, hipMemsetAsync(c->lts_st, 0, sizeof(StepState), c->stream));
  HIPCHK(c, hipMemsetAsync(c->lts_ring, 0, 2 * sizeof(double), c->stream));
  for (void* p : {c->lts_s, c->lts_w, c->lts_qa, c->lts_qb, c->lts_ep, c->lts_x[0], c->lts_x[1]})
    if (p) HIPCHK(c, hipMemsetAsync(p, 0, pb, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->lts_p = sub ? substeps : 1;
  c->lts_dt = dt_coarse;
  c->lts_every = energy_every;
  c->lts = true;
  if (!sub)
    for (LtsBox& x : c->lts_tbox) x.on = x.refined = 0;
  sbp_status st = lts_lists(c);
  if (st != SBP_OK) return st;
  if (sub || track) {
    // E^{-1} = E^0 - dt A H^{-1/2} (on the near boxes; everywhere for the
    // energy): the scratch state (E = 0, H = H^{-1/2}) after one unit step
    // on all tiles holds A H^{-1/2}; the scratch state and its face buffers
    // are cleared again afterwards
    const bool f64 = c->prec == SBP_FP64;
    void* M = pool_at(c, c->nstep);
    const int threads = c->tx * c->ty;
    auto phase = [&](int op, int nmode, const Tile* tiles, int ntiles) {
      return f64 ? lts_phase<double>(op, nmode, 0, M, c->lts_s, nullptr, nullptr, nullptr, nullptr, c->lts_ep, 0.0,
                                     dt_coarse, tiles, ntiles, c->d_blocks, c->lts_boxes, threads, c->cz, c->stream)
                 : lts_phase<float>(op, nmode, 0, M, c->lts_s, nullptr, nullptr, nullptr, nullptr, c->lts_ep, 0.0,
                                    dt_coarse, tiles, ntiles, c->d_blocks, c->lts_boxes, threads, c->cz, c->stream);
    };
    HIPCHK(c, phase(-1, 2, c->d_tiles_bare, c->ntiles));
    if ((st = lts_apply(c, true)) != SBP_OK) return st;
    if (sub) HIPCHK(c, phase(4, -1, c->d_near, c->nnear));
    if (track)
      HIPCHK(c, f64 ? lts_whole<double>(1, nb, M, c->lts_x[1], c->lts_s, dt_coarse, c->d_blocks, c->stream)
                    : lts_whole<float>(1, nb, M, c->lts_x[1], c->lts_s, dt_coarse, c->d_blocks, c->stream));
    HIPCHK(c, hipMemsetAsync(c->lts_s, 0, pb, c->stream));
    HIPCHK(c, hipMemsetAsync(c->lts_face, 0, c->face_elems * sizeof(double), c->stream));
  }
  return SBP_OK;
}

sbp_status sbp_lts_step(sbp_ctx* c, long nsteps) {
  if (!c) return SBP_EINVAL;
  if (!c->lts) return fail(c, SBP_ESTATE, "sbp_lts_step before sbp_lts_start");
  if (nsteps < 0) return fail(c, SBP_EINVAL, "negative step count");
  if (nsteps == 0) return SBP_OK;
  HIPCHK(c, hipSetDevice(c->device));
  if (c->near_dirty) {
    const sbp_status st = lts_lists(c);
    if (st != SBP_OK) return st;
  }
  const bool f64 = c->prec == SBP_FP64;
  const int nb = (int)c->blocks.size(), p = c->lts_p, threads = c->tx * c->ty;
  const double dt = c->lts_dt, tau = dt / p, tau2 = tau * tau;
  const long K = c->lts_every;
  const KArgs ka = kargs(c);
  auto phase = [&](int op, int nmode, int last, void* M, const void* qm, const void* qp, void* qo) {
    return f64 ? lts_phase<double>(op, nmode, last, M, c->lts_s, c->lts_w, qm, qp, qo, c->lts_ep, tau2, dt, c->d_near,
                                   c->nnear, c->d_blocks, c->lts_boxes, threads, c->cz, c->stream)
               : lts_phase<float>(op, nmode, last, M, c->lts_s, c->lts_w, qm, qp, qo, c->lts_ep, tau2, dt, c->d_near,
                                  c->nnear, c->d_blocks, c->lts_boxes, threads, c->cz, c->stream);
  };
  auto copy = [&](const void* M, void* X) {
    return f64 ? lts_whole<double>(0, nb, M, X, nullptr, 0.0, c->d_blocks, c->stream)
               : lts_whole<float>(0, nb, M, X, nullptr, 0.0, c->d_blocks, c->stream);
  };
  auto energy = [&](const void* M, const void* X, const void* Y) {
    const double scale = 0.5 / (dt * dt);
    return f64 ? lts_energy<double>(M, X, Y, scale, c->d_tiles_bare, c->ntiles, c->d_blocks, c->mat[0], kEps0,
                                    threads, c->cz, c->lts_part, c->stream)
               : lts_energy<float>(M, X, Y, scale, c->d_tiles_bare, c->ntiles, c->d_blocks, c->mat[0], kEps0,
                                   threads, c->cz, c->lts_part, c->stream);
  };
  sbp_status st;
  // the scratch state of the first operator step: E = (I - P) E^n
  if (p > 1) HIPCHK(c, phase(-1, 0, 0, pool_at(c, c->nstep), nullptr, nullptr, nullptr));
  for (long s = 0; s < nsteps; ++s) {
    const long long n = c->nstep;
    void* M = pool_at(c, n);  // E^n, H^{n-1/2} (the two-pass step keeps one pool)
    if (p > 1) {
      // w = L (I - P) E^n; q_1; then q_{m+1} from q_m, q_{m-1} (q_m in
      // lts_qa for odd m, lts_qb for even m > 0); the last substep leaves
      // E^{n+1} in lts_w
      if ((st = lts_apply(c, false)) != SBP_OK) return st;
      HIPCHK(c, phase(0, 1, 0, M, nullptr, nullptr, nullptr));
      if ((st = lts_apply(c, false)) != SBP_OK) return st;
      HIPCHK(c, phase(1, 1, 0, M, nullptr, nullptr, c->lts_qa));
      for (int m = 1; m < p; ++m) {
        void* qm = (m & 1) ? c->lts_qa : c->lts_qb;
        const void* qp = m == 1 ? M : ((m & 1) ? c->lts_qb : c->lts_qa);
        void* qo = (m & 1) ? c->lts_qb : c->lts_qa;
        const bool last = m == p - 1;
        if ((st = lts_apply(c, false)) != SBP_OK) return st;
        HIPCHK(c, phase(2, last ? -1 : 1, last ? 1 : 0, M, qm, qp, qo));
      }
    }
    // copies of E^n for the energy of this step or the next
    const bool form = K > 0 && n % K == 0;
    if (K > 0 && (form || (n + 1) % K == 0)) HIPCHK(c, copy(M, c->lts_x[n & 1]));
    // the ordinary step of length dt on the blocks that are not refined
    KArgs a = ka;
    a.blocks = c->lts_cblocks;
    a.dt = dt;
    if (p > 1) {
      a.tiles = c->d_far;
      const StepLists far{c->fk_t0x, c->fk_t1x, c->d_fwg[0], c->d_fwg[1], c->nfwg[0], c->nfwg[1], true};
      st = enqueue_step_on(c, a, false, &far);
    } else {
      a.tiles = c->d_tiles_bare;
      st = enqueue_step_on(c, a, false);
    }
    if (st != SBP_OK) return st;
    // the scheme's E^{n+1} on the near boxes, and the next step's scratch state
    if (p > 1) HIPCHK(c, phase(3, s + 1 < nsteps ? 0 : -1, 0, M, nullptr, nullptr, nullptr));
    double* slot = ka.energy + (int)(n % ka.ecap);
    if (form) {
      HIPCHK(c, energy(M, c->lts_x[(n + 1) & 1], c->lts_x[n & 1]));
      HIPCHK(c, lts_store(c->lts_part, c->ntiles, slot, c->stream));
    } else {
      HIPCHK(c, lts_store(c->lts_part, 0, slot, c->stream));
    }
    c->nstep += 1;
  }
  return SBP_OK;
}

sbp_status sbp_lts_info(const sbp_ctx* c, long out[4]) {
  if (!c || !out) return SBP_EINVAL;
  if (!c->lts) return SBP_ESTATE;
  out[0] = c->nnear;
  out[1] = c->ntiles;
  out[2] = out[3] = 0;
  for (size_t b = 0; b < c->blocks.size(); ++b) {
    const HostBlock& hb = c->blocks[b];
    const LtsBox& x = c->lts_hbox[b];
    if (x.on) out[2] += (long)(x.hi[0] - x.lo[0] + 1) * (x.hi[1] - x.lo[1] + 1) * (x.hi[2] - x.lo[2] + 1);
    out[3] += (long)(hb.n[0] + 2) * (hb.n[1] + 2) * (hb.n[2] + 2);
  }
  return SBP_OK;
}

sbp_status sbp_steps_done(const sbp_ctx* c, long* n) {
  if (!c || !n) return SBP_EINVAL;
  *n = (long)c->nstep;
  return SBP_OK;
}

sbp_status sbp_field_shape(const sbp_ctx* c, int block, sbp_comp comp, int shape[3]) {
  if (!c || !shape) return SBP_EINVAL;
  if (!check_block(c, block) || comp < SBP_EX || comp > SBP_HZ) return SBP_EINVAL;
  for (int a = 0; a < 3; ++a) shape[a] = comp_dim(c->blocks[block], comp, a);
  return SBP_OK;
}

sbp_status sbp_read_field(sbp_ctx* c, int block, sbp_comp comp, double* dst, size_t count) {
  if (!c || !dst) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "read_field before finalize");
  if (!check_block(c, block) || comp < SBP_EX || comp > SBP_HZ) return fail(c, SBP_EINVAL, "bad block or component");
  int s[3];
  sbp_field_shape(c, block, comp, s);
  if (count < (size_t)s[0] * s[1] * s[2]) return fail(c, SBP_EINVAL, "destination too small");
  const DevBlock& d = c->hblocks[block];
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const char* src = (const char*)pool_at(c, c->nstep) + (size_t)(d.foff + comp * d.csz) * elem_size(c);
  if (c->prec == SBP_FP64) {
    std::vector<double> box(d.csz);
    HIPCHK(c, hipMemcpy(box.data(), src, d.csz * 8, hipMemcpyDeviceToHost));
    extract(box, d, s, dst);
  } else {
    std::vector<float> box(d.csz);
    HIPCHK(c, hipMemcpy(box.data(), src, d.csz * 4, hipMemcpyDeviceToHost));
    extract(box, d, s, dst);
  }
  return SBP_OK;
}

sbp_status sbp_write_field(sbp_ctx* c, int block, sbp_comp comp, const double* srcp, size_t count) {
  if (!c || !srcp) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "write_field before finalize");
  if (c->lts) return fail(c, SBP_ESTATE, "the context steps by local time stepping (sbp_lts_step)");
  if (!check_block(c, block) || comp < SBP_EX || comp > SBP_HZ) return fail(c, SBP_EINVAL, "bad block or component");
  int s[3];
  sbp_field_shape(c, block, comp, s);
  if (count < (size_t)s[0] * s[1] * s[2]) return fail(c, SBP_EINVAL, "source too small");
  const DevBlock& d = c->hblocks[block];
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  char* dstp = (char*)pool_at(c, c->nstep) + (size_t)(d.foff + comp * d.csz) * elem_size(c);
  if (c->prec == SBP_FP64) {
    std::vector<double> box(d.csz, 0.0);
    insert(box, d, s, srcp);
    HIPCHK(c, hipMemcpy(dstp, box.data(), d.csz * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> box(d.csz, 0.0f);
    insert(box, d, s, srcp);
    HIPCHK(c, hipMemcpy(dstp, box.data(), d.csz * 4, hipMemcpyHostToDevice));
  }
  return SBP_OK;
}

sbp_status sbp_read_energy(sbp_ctx* c, long first, long count, double* dst) {
  if (!c || (!dst && count > 0)) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "read_energy before finalize");
  if (first < 0 || count < 0 || first + count > c->nstep || first <= c->nstep - c->history)
    return fail(c, SBP_ERANGE, "energy samples not available");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<double> ring(c->history);
  HIPCHK(c, hipMemcpy(ring.data(), c->d_energy, ring.size() * 8, hipMemcpyDeviceToHost));
  for (long q = 0; q < count; ++q) dst[q] = ring[(first + q) % c->history];
  StepState st;
  HIPCHK(c, hipMemcpy(&st, c->d_st, sizeof(st), hipMemcpyDeviceToHost));
  if (st.flags & 1) return fail(c, SBP_EUNSTABLE, "non-finite energy");
  return SBP_OK;
}

sbp_status sbp_read_probe(sbp_ctx* c, int id, long first, long count, double* dst) {
  if (!c || (!dst && count > 0)) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "read_probe before finalize");
  if (id < 0 || id >= (int)c->prbs.size()) return fail(c, SBP_EINVAL, "bad probe id");
  if (first < 0 || count < 0 || first + count > c->nstep || first < c->nstep - c->history)
    return fail(c, SBP_ERANGE, "probe samples not available");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<double> ring(c->history);
  HIPCHK(c, hipMemcpy(ring.data(), c->d_probes + (size_t)c->probe_order[id] * c->history, ring.size() * 8,
                      hipMemcpyDeviceToHost));
  for (long q = 0; q < count; ++q) dst[q] = ring[(first + q) % c->history];
  return SBP_OK;
}

sbp_status sbp_state_bytes(const sbp_ctx* c, size_t* bytes) {
  if (!c || !bytes) return SBP_EINVAL;
  if (!c->finalized) return SBP_ESTATE;
  // fields, step state, CPML psi, TF/SF incident line
  *bytes = c->pool_elems * elem_size(c) + 256 + c->psi_elems * elem_size(c) + line_bytes(c);
  return SBP_OK;
}

sbp_status sbp_save_state(sbp_ctx* c, void* dev_buf, size_t bytes) {
  if (c && c->lts) return fail(c, SBP_ESTATE, "the saved state does not hold local time stepping's E^{n-1}");
  if (!c || !dev_buf) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "save_state before finalize");
  size_t need;
  sbp_state_bytes(c, &need);
  if (bytes < need) return fail(c, SBP_EINVAL, "state buffer too small");
  HIPCHK(c, hipMemcpyAsync(dev_buf, pool_at(c, c->nstep), c->pool_elems * elem_size(c), hipMemcpyDeviceToDevice,
                           c->stream));
  HIPCHK(c, hipMemcpyAsync((char*)dev_buf + c->pool_elems * elem_size(c), c->d_st, sizeof(StepState),
                           hipMemcpyDeviceToDevice, c->stream));
  const size_t po = c->pool_elems * elem_size(c) + 256;
  if (c->psi_elems)
    HIPCHK(c, hipMemcpyAsync((char*)dev_buf + po, c->d_psi, c->psi_elems * elem_size(c), hipMemcpyDeviceToDevice,
                             c->stream));
  if (c->tf_on)
    HIPCHK(c, hipMemcpyAsync((char*)dev_buf + po + c->psi_elems * elem_size(c), c->d_line, line_bytes(c),
                             hipMemcpyDeviceToDevice, c->stream));
  return SBP_OK;
}

sbp_status sbp_load_state(sbp_ctx* c, const void* dev_buf, size_t bytes) {
  if (c && c->lts) return fail(c, SBP_ESTATE, "the saved state does not hold local time stepping's E^{n-1}");
  if (!c || !dev_buf) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "load_state before finalize");
  size_t need;
  sbp_state_bytes(c, &need);
  if (bytes < need) return fail(c, SBP_EINVAL, "state buffer too small");
  StepState st;
  HIPCHK(c, hipMemcpyAsync(&st, (const char*)dev_buf + c->pool_elems * elem_size(c), sizeof(StepState),
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpyAsync(pool_at(c, st.step), dev_buf, c->pool_elems * elem_size(c), hipMemcpyDeviceToDevice,
                           c->stream));
  const size_t po = c->pool_elems * elem_size(c) + 256;
  if (c->psi_elems)
    HIPCHK(c, hipMemcpyAsync(c->d_psi, (const char*)dev_buf + po, c->psi_elems * elem_size(c),
                             hipMemcpyDeviceToDevice, c->stream));
  if (c->tf_on)
    HIPCHK(c, hipMemcpyAsync(c->d_line, (const char*)dev_buf + po + c->psi_elems * elem_size(c), line_bytes(c),
                             hipMemcpyDeviceToDevice, c->stream));
  st.flags = 0;
  HIPCHK(c, hipMemcpyAsync(c->d_st, &st, sizeof(st), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->nstep = st.step;
  return SBP_OK;
}

sbp_status sbp_use_graph(sbp_ctx* c, int steps) {
  if (!c || steps < 0) return SBP_EINVAL;
  if (steps > 0 && c->stream == nullptr)
    return fail(c, SBP_EINVAL, "graph capture needs a non-default stream");
  drop_graph(c);
  c->graph_steps = steps;
  return SBP_OK;
}

sbp_status sbp_last_step_ms(sbp_ctx* c, double* ms) {
  if (!c || !ms) return SBP_EINVAL;
  if (!c->timed) return fail(c, SBP_ESTATE, "no timed step yet");
  HIPCHK(c, hipEventSynchronize(c->ev1));
  float f = 0.0f;
  HIPCHK(c, hipEventElapsedTime(&f, c->ev0, c->ev1));
  *ms = f;
  return SBP_OK;
}

sbp_status sbp_profile(sbp_ctx* c, int enable) {
  if (!c) return SBP_EINVAL;
  c->profile = enable != 0;
  return SBP_OK;
}

sbp_status sbp_kernel_ms(sbp_ctx* c, double out[3]) {
  if (!c || !out) return SBP_EINVAL;
  if (!c->profile || c->kev_used < 6) return fail(c, SBP_ESTATE, "no profiled step");
  HIPCHK(c, hipEventSynchronize(c->kev[c->kev_used - 1]));
  double acc[3] = {0.0, 0.0, 0.0};
  const int steps = c->kev_used / 6;
  for (int s = 0; s < steps; ++s)
    for (int q = 0; q < 3; ++q) {
      float ms = 0.0f;
      HIPCHK(c, hipEventElapsedTime(&ms, c->kev[6 * s + 2 * q], c->kev[6 * s + 2 * q + 1]));
      acc[q] += ms;
    }
  for (int q = 0; q < 3; ++q) out[q] = acc[q] / steps;
  return SBP_OK;
}

sbp_status sbp_autotune(sbp_ctx* c, int steps_per_trial, double* best_ms) {
  if (!c) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "autotune before finalize");
  if (c->lts) return fail(c, SBP_ESTATE, "the context steps by local time stepping (sbp_lts_step)");
  if (steps_per_trial < 1) steps_per_trial = 5;
  size_t bytes;
  sbp_state_bytes(c, &bytes);
  void* save = dalloc(c, bytes);
  if (!save) return fail(c, SBP_ENOMEM, "autotune snapshot allocation failed");
  sbp_status st = sbp_save_state(c, save, bytes);
  if (st != SBP_OK) return st;
  const int keep[4] = {c->tx, c->ty, c->cz, c->wgs};
  const bool prof = c->profile;
  const int gsteps = c->graph_steps;
  c->profile = false;
  drop_graph(c);
  c->graph_steps = 0;
  int dev_cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) dev_cus = prop.multiProcessorCount;
  struct Cand { int tx, ty, cz, wg; };
  std::vector<Cand> cand;
  // threads per tile x planes per tile, one workgroup per tile; then the
  // kept shape with resident workgroups looping over the tile list
  const int ths[3] = {64, 128, 256};
  const int czs[5] = {1, 2, 4, 8, 16};
  for (int t : ths)
    for (int cz : czs) cand.push_back({t, 1, cz, 0});
  cand.push_back({keep[0], keep[1], keep[2], dev_cus * 8});
  cand.push_back({keep[0], keep[1], keep[2], dev_cus * 16});
  double best = 1e300;
  Cand win{keep[0], keep[1], keep[2], keep[3]};
  for (const Cand& k : cand) {
    st = sbp_set_launch(c, k.tx, k.ty, k.cz, k.wg);
    if (st != SBP_OK) break;
    if ((st = sbp_load_state(c, save, bytes)) != SBP_OK) break;
    if ((st = sbp_step(c, 1)) != SBP_OK) break;  // warm-up
    if ((st = sbp_step(c, steps_per_trial)) != SBP_OK) break;
    double ms = 0.0;
    if ((st = sbp_last_step_ms(c, &ms)) != SBP_OK) break;
    ms /= steps_per_trial;
    if (ms < best) {
      best = ms;
      win = k;
    }
  }
  sbp_status st2 = sbp_set_launch(c, win.tx, win.ty, win.cz, win.wg);
  sbp_status st3 = sbp_load_state(c, save, bytes);
  dfree(c, save);
  c->profile = prof;
  c->graph_steps = gsteps;
  if (st != SBP_OK) return st;
  if (st2 != SBP_OK) return st2;
  if (st3 != SBP_OK) return st3;
  if (best_ms) *best_ms = best;
  return SBP_OK;
}

sbp_status sbp_adjoint(sbp_ctx* c, int block, long nsteps, const int region[6], long ckpt_every, double* J_out,
                       double* grad_eps_dev) {
  if (!c || !region || !J_out) return SBP_EINVAL;
  if (!c->finalized) return fail(c, SBP_ESTATE, "adjoint before finalize");
  if (c->lts) return fail(c, SBP_ESTATE, "the context steps by local time stepping (sbp_lts_step)");
  if (!check_block(c, block)) return fail(c, SBP_EINVAL, "bad block");
  if (nsteps < 1) return fail(c, SBP_EINVAL, "nsteps must be >= 1");
  const HostBlock& hb = c->blocks[block];
  for (int a = 0; a < 3; ++a)
    if (region[2 * a] < 0 || region[2 * a + 1] > hb.n[a] || region[2 * a] >= region[2 * a + 1])
      return fail(c, SBP_EINVAL, "region must be a non-empty cell box inside the block");
  for (const HostBlock& b : c->blocks) {
    bool lossy = false;
    for (double v : b.sig) lossy = lossy || v != 0.0;
    for (int f = 0; f < 6; ++f) lossy = lossy || (b.iface[f] < 0 && (b.faces[f] == SBP_ABC1 || b.faces[f] == SBP_CPML));
    if (lossy) return fail(c, SBP_EINVAL, "the adjoint covers lossless blocks (no conductivity, no absorbing faces)");
    if (b.tfsf) return fail(c, SBP_EINVAL, "the adjoint does not cover TF/SF injection");
  }
  long K = ckpt_every > 0 ? ckpt_every : (long)std::ceil(std::sqrt((double)nsteps));
  if (K > nsteps) K = nsteps;
  const long nck = (nsteps + K - 1) / K;
  const bool f64 = c->prec == SBP_FP64;
  const size_t pb = c->pool_elems * elem_size(c);
  const size_t sb = pb + sizeof(StepState);
  const DevBlock& d = c->hblocks[block];
  const size_t gsz = 3 * (size_t)d.csz;
  const size_t ncell = (size_t)hb.n[0] * hb.n[1] * hb.n[2];
  HIPCHK(c, hipSetDevice(c->device));
  drop_graph(c);
  if (!grad_eps_dev) {
    // the objective alone: the forward run with J summed after every step
    double* Jd = (double*)dalloc(c, sizeof(double));
    if (!Jd) return fail(c, SBP_ENOMEM, "adjoint buffer allocation failed");
    auto run_j = [&]() -> sbp_status {
      HIPCHK(c, hipMemsetAsync(Jd, 0, sizeof(double), c->stream));
      const long long n0 = c->nstep;
      HIPCHK(c, launch_sources(kargs(c), c->stream));
      for (long n = 0; n < nsteps; ++n) {
        const sbp_status s2 = enqueue_step(c, false);
        if (s2 != SBP_OK) return s2;
        void* now = pool_at(c, n0 + n + 1);
        HIPCHK(c, f64 ? launch_adj_objective<double>(now, c->d_blocks, block, region, c->dt, Jd, c->stream)
                      : launch_adj_objective<float>(now, c->d_blocks, block, region, c->dt, Jd, c->stream));
      }
      HIPCHK(c, hipMemcpyAsync(J_out, Jd, sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      return SBP_OK;
    };
    const sbp_status sj = run_j();
    dfree(c, Jd);
    if (sj == SBP_OK) c->nstep += nsteps;
    return sj;
  }
  // buffers: checkpoints, one segment of forward states, the adjoint state
  // (pool, face buffers, step counter, one-slot energy / probe rings), dJ/dCb
  std::vector<void*> tmp;
  auto take = [&](size_t bytes) {
    void* p = dalloc(c, bytes);
    if (p) tmp.push_back(p);
    return p;
  };
  char* ck = (char*)take(nck * sb);
  char* seg = (char*)take((K + 1) * pb);
  char* fin = (char*)take(sb);
  void* apool = take(pb);
  void* apool2 = c->pool2 != c->pool ? take(pb) : apool;
  double* aface = (double*)take(c->face_elems * sizeof(double));
  StepState* ast = (StepState*)take(sizeof(StepState));
  double* ering = (double*)take(2 * sizeof(double));
  double* pring = (double*)take(std::max<size_t>(c->prbs.size(), 1) * sizeof(double));
  double* G = (double*)take(gsz * sizeof(double));
  double* Jd = (double*)take(sizeof(double));
  auto release = [&]() {
    for (void* p : tmp) dfree(c, p);
  };
  if (!ck || !seg || !fin || !apool || !apool2 || !aface || !ast || !ering || !pring || !G || !Jd) {
    release();
    return fail(c, SBP_ENOMEM, "adjoint buffer allocation failed");
  }
  sbp_status st = SBP_OK;
  auto run = [&]() -> sbp_status {
    HIPCHK(c, hipMemsetAsync(apool, 0, pb, c->stream));
    if (apool2 != apool) HIPCHK(c, hipMemsetAsync(apool2, 0, pb, c->stream));
    HIPCHK(c, hipMemsetAsync(aface, 0, c->face_elems * sizeof(double), c->stream));
    HIPCHK(c, hipMemsetAsync(ast, 0, sizeof(StepState), c->stream));
    HIPCHK(c, hipMemsetAsync(G, 0, gsz * sizeof(double), c->stream));
    // the step kernels write valid nodes only: the segment's other nodes stay zero
    HIPCHK(c, hipMemsetAsync(seg, 0, (K + 1) * pb, c->stream));
    HIPCHK(c, hipMemsetAsync(Jd, 0, sizeof(double), c->stream));
    HIPCHK(c, hipMemsetAsync(grad_eps_dev, 0, ncell * sizeof(double), c->stream));
    // forward: N steps from the current state n0, checkpoints every K steps, J
    const long long n0 = c->nstep;
    HIPCHK(c, launch_sources(kargs(c), c->stream));
    for (long n = 0; n < nsteps; ++n) {
      if (n % K == 0) {
        char* dst = ck + (size_t)(n / K) * sb;
        HIPCHK(c, hipMemcpyAsync(dst, pool_at(c, n0 + n), pb, hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(dst + pb, c->d_st, sizeof(StepState), hipMemcpyDeviceToDevice, c->stream));
      }
      sbp_status s2 = enqueue_step(c, false);
      if (s2 != SBP_OK) return s2;
      void* now = pool_at(c, n0 + n + 1);
      HIPCHK(c, f64 ? launch_adj_objective<double>(now, c->d_blocks, block, region, c->dt, Jd, c->stream)
                    : launch_adj_objective<float>(now, c->d_blocks, block, region, c->dt, Jd, c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(fin, pool_at(c, n0 + nsteps), pb, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(fin + pb, c->d_st, sizeof(StepState), hipMemcpyDeviceToDevice, c->stream));
    // adjoint state p^N = Cb / w_E dJ/dE^N, r^{N+1/2} = 0
    HIPCHK(c, f64 ? launch_adj_source<double>(apool, fin, c->d_blocks, c->mat[0], block, region, c->dt, c->stream)
                  : launch_adj_source<float>(apool, fin, c->d_blocks, c->mat[0], block, region, c->dt, c->stream));
    // the forward replays write their energy / probe samples to one-slot
    // scratch rings (the context's rings keep the forward samples); the
    // adjoint state has its own pool, face buffers and step counter, and
    // tiles without source / probe flags
    KArgs fwd = kargs(c);
    fwd.energy = ering;
    fwd.ecap = 1;
    fwd.probes = pring;
    fwd.pcap = 1;
    KArgs adj = fwd;
    adj.pool = apool;  // adjoint step m reads apool (m even) or apool2 (m odd)
    adj.pool2 = apool2;
    adj.face = aface;
    adj.st = ast;
    adj.tiles = c->d_tiles_bare;
    adj.ftiles = c->d_ftiles_bare;
    adj.nsrc = 0;
    long m = 0;  // adjoint steps taken
    for (long sgi = nck - 1; sgi >= 0; --sgi) {
      const long a = sgi * K, b = std::min(a + K, nsteps);
      const char* src = ck + (size_t)sgi * sb;
      // segment slot s holds the state at step a + s: the replay of step n
      // reads slot n - a and writes slot n + 1 - a (the step kernels take
      // their input and output pools by the parity of the step index)
      HIPCHK(c, hipMemcpyAsync(seg, src, pb, hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(c, hipMemcpyAsync(c->d_st, src + pb, sizeof(StepState), hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(c, launch_sources(fwd, c->stream));
      for (long n = a; n < b; ++n) {
        KArgs f = fwd;
        void* in = seg + (size_t)(n - a) * pb;
        void* out = seg + (size_t)(n + 1 - a) * pb;
        f.pool = ((n0 + n) & 1) ? out : in;
        f.pool2 = ((n0 + n) & 1) ? in : out;
        sbp_status s2 = enqueue_step_on(c, f, false);
        if (s2 != SBP_OK) return s2;
      }
      for (long n = b - 1; n >= a; --n) {
        const char* enew = seg + (size_t)(n + 1 - a) * pb;
        const char* eold = seg + (size_t)(n - a) * pb;
        const char* acur = (const char*)((m & 1) ? apool2 : apool);
        const size_t eoff = (size_t)d.foff * elem_size(c);  // the block's Ex, Ey, Ez: 3 csz values from foff
        HIPCHK(c, f64 ? launch_adj_grad<double>(acur + eoff, enew + eoff, eold + eoff, 3LL * d.csz, G, c->stream)
                      : launch_adj_grad<float>(acur + eoff, enew + eoff, eold + eoff, 3LL * d.csz, G, c->stream));
        sbp_status s2 = enqueue_step_on(c, adj, false);
        if (s2 != SBP_OK) return s2;
        ++m;
        void* anext = (m & 1) ? apool2 : apool;
        if (n >= 1)
          HIPCHK(c, f64 ? launch_adj_source<double>(anext, eold, c->d_blocks, c->mat[0], block, region, c->dt,
                                                    c->stream)
                        : launch_adj_source<float>(anext, eold, c->d_blocks, c->mat[0], block, region, c->dt,
                                                   c->stream));
      }
    }
    HIPCHK(c, f64 ? launch_adj_cells<double>(c->d_blocks, c->mat[0], block, G, grad_eps_dev, c->stream)
                  : launch_adj_cells<float>(c->d_blocks, c->mat[0], block, G, grad_eps_dev, c->stream));
    // back to the state after the forward run
    HIPCHK(c, hipMemcpyAsync(pool_at(c, n0 + nsteps), fin, pb, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_st, fin + pb, sizeof(StepState), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(J_out, Jd, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SBP_OK;
  };
  st = run();
  (void)hipStreamSynchronize(c->stream);
  release();
  if (st != SBP_OK) return st;
  c->nstep += nsteps;
  return SBP_OK;
}

const char* sbp_last_error(const sbp_ctx* c) { return c ? c->err.c_str() : "null context"; }

void sbp_destroy(sbp_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  drop_graph(c);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->kev) (void)hipEventDestroy(e);
  std::vector<void*> a = c->allocs;
  for (void* p : a) dfree(c, p);
  delete c;
}

}  // extern "C"
