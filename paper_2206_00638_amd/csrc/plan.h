// Device-side plan of the SBP-SAT FDTD step: per-block descriptors, tiles,
// sources, probes and interface gather jobs.  Plain structs shared by the
// host plan (api.hip) and the kernels (step.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbp {

enum Comp { EX = 0, EY, EZ, HX, HY, HZ };

// One boundary-closure row of D+ or D- along an axis (Appendix), with the
// SAT row changes of Section III folded in.  The row reads the three
// consecutive nodes row+s .. row+s+2 with coefficients c (already / h); on an
// interface face the own boundary coefficient is zero and cn (already / h)
// multiplies the neighbour value gathered into the face buffer.
struct Row {
  int s;
  int nbr;  // 1: add cn * neighbour face value
  double c[3];
  double cn;
};

// Rows of D+ held in the table: 0, 1, n-1, n.  Rows of D-: 0, 1, 2, n-1, n, n+1.
// Plain blocks whose per-cell permittivity takes at most kCellTab distinct
// values (in the field precision) hold a byte index per cell and a table.
constexpr int kCellTab = 64;
constexpr int DP_ROWS = 4;
constexpr int DM_ROWS = 6;

enum MatFlags { MAT_EPS = 1, MAT_MU = 2, MAT_SIG = 4 };

struct DevBlock {
  int n[3];
  int mat;              // MatFlags: which per-cell arrays exist
  long long sx, sxy;    // node-box strides: node (i,j,k) at i + sx*j + sxy*k; sxy = sx(ny+2) rounded up to 64
  long long csz;        // component stride sxy (nz+2)
  long long foff;       // pool offset of component 0; component c at foff + c*csz
  long long coff;       // offset of this block's cells in the material arrays
  double h[3], ih[3];
  double eps_r0, mu_r0, sig0;  // uniform values where no per-cell array
  Row dp[3][DP_ROWS];
  Row dm[3][DM_ROWS];
  int abc_mask;         // bit f: face f absorbing
  int iface_mask;       // bit f: face f coupled to another block
  int pml_stride;       // absorbing layers: entries per profile (max n + 2), 0 if none
  long long pml_off;    // profile table offset: (b, c, 1/kappa) of axis a, grid g
                        // ("+" 0, "-" 1), quantity q at pml_off + ((a*2+g)*3+q)*stride + idx
  long long psi_off;    // psi arrays of the layers: slot s (0-5 H terms, 6-11 E terms)
                        // of node offset o at psi_off + s*csz + o
  long long fboff[6];   // face-buffer offset (doubles): E slot 0,1 then H slot 0,1
  long long fsz[6];     // nodes per slot of the face buffer (node-box face)
  int src0, nsrc, prb0, nprb;
  // fast-path constants (interior nodes), in fp64; cast to the field type
  double db_u;    // dt / (mu0 mu_r0): H update with uniform permeability
  double cb_u;    // dt / (eps0 eps_r0): E update with uniform permittivity, lossless
  double dte0x4;  // 4 dt / eps0: Cb = dte0x4 / (sum of the four cell eps_r)
  double hdte0;   // dt / (2 eps0): loss factor b = hdte0 * sigma_sum / eps_sum
  double dtm0x2;  // 2 dt / mu0: Db = dtm0x2 / (sum of the two cell mu_r)
  double ke, kh;  // 1/2 eps0 hx hy hz, 1/2 mu0 hx hy hz (energy of an interior node)
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Norm weights / h (Appendix P+, P-) of node r on an axis of n cells.
__device__ __forceinline__ float wp1(int n, int r) { return (r == 0 || r == n) ? 0.5f : 1.0f; }
__device__ __forceinline__ float wm1(int n, int r) {
  if (r == 0 || r == n + 1) return 0.5f;
  if (r == 1 || r == n) return 0.25f;
  if (r == 2 || r == n - 1) return 1.25f;
  return 1.0f;
}

// Sum over a wave (64 lanes); lane 0 holds the total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// A tile is `threads` consecutive nodes q0 .. q0+threads-1 of the flattened
// (i fastest) xy node plane of one block, over the planes z0 .. z0+cz-1: each
// thread walks one node column through the cz planes.  pad holds flags:
// bit 0 = a source, bit 1 = a probe lies in the tile.
struct Tile {
  int block, q0, z0, pad;
};

// A tile of the one-pass step: a 32 x 8 window of node columns of one
// block's xy plane starting at (i0, j0), on which H^{n+1/2} is formed, and
// its owned part [olx, ohx] x [oly, ohy] x planes [z0, z1], on which H and E
// are written (the unowned columns supply neighbour values of H only).
// flags: bit 0 = a source, bit 1 = a probe lies in the owned part.
constexpr int FX = 32, FY = 8;
struct FTile {
  int block, i0, j0, olx, ohx, oly, ohy, z0, z1, flags;
};

struct Source {
  int comp, i, j, k;
  int wave, pad;
  double tw, t0, f0, amp;
};

struct Probe {
  int comp, i, j, k;
};

// Interface gather: fills face-buffer slot `slot` (E or H) of (block, face)
// from the neighbour's face through per-axis tap tables.
constexpr int MAX_TAPS = 8;
struct Taps {
  int start, count;
  double w[MAX_TAPS];
};
struct FaceJob {
  int block, face, is_h, slot;
  int comp;             // component gathered
  int nb;               // neighbour block
  int nb2;              // second source block (periodic faces of complex
                        // fields: the other part), or -1
  double w1, w2;        // value = w1 * (nb's face) + w2 * (nb2's face)
  int nb_idx;           // face-normal node index of the neighbour face
  int unit;             // 1: same mesh on both tangential axes (no taps)
  int t_axis[2];        // tangential axes (ascending)
  int ext[2];           // own face-node extents along the tangential axes
  long long taps_off[2];  // offsets into the tap table for each tangential axis
};

// One workgroup of a face gather: job index and first face node (a job's
// nodes are split into runs of 256, one per workgroup).
struct GatherWG {
  int job, first;
};

struct StepState {
  long long step;       // index n of the next step
  int flags;            // bit 0: non-finite energy seen
};


// Total-field / scattered-field injection (one box per context): the
// block, the cell box [lo, hi] per axis, the propagation axis (+axis), the
// incident E and H components (0-2), and the incident line (fp64, E at "+"
// index i in e1[i + margin], H at (i + 1/2) h in h1[i + margin]).
struct TfDesc {
  double* e1;
  double* h1;
  double ch, ce;  // line coefficients: dt s_H / (mu0 h), dt s_E / (eps0 h), s the signs of
                  // d_axis in the H and E equations of the incident pair
  int block, axis, ep, hq, margin, len;
  int src;   // line index of the incident soft source
  int sidx;  // its slot in srcval (after the point sources of every block)
  int lo[3], hi[3];
  // the two curl terms that difference the incident E component (H side)
  // and the incident H component (E side): component, difference axis, sign
  int h_comp[2], h_ax[2], e_comp[2], e_ax[2];
  double h_sg[2], e_sg[2];
};

// Arguments of the step kernels (one struct, passed by value).
struct KArgs {
  const DevBlock* blocks;
  const Tile* tiles;
  const FTile* ftiles;
  int ntiles;
  int cz;
  int order;   // tile walk: 0 = dispatch order, 1 = contiguous ranges per XCD
  void* pool;   // field pools: step n reads pool (n even) or pool2 (n odd)
  void* pool2;  // and writes the other one
  const void* mat_eps;
  const unsigned char* mat_idx;  // byte index per cell of the tabled blocks (kind bit 5)
  const void* mat_tab;           // their tables: block b's kCellTab values at b * kCellTab
  const void* mat_mu;
  const void* mat_sig;
  const double* face;
  const void* pml_prof;  // absorbing-layer profiles (field type)
  void* psi;             // absorbing-layer recursion variables (field type)
  const Source* src;
  double* srcval;  // current density of each source at (n+1/2) dt of the step
  int nsrc;        // sources over all blocks
  const Probe* prb;
  double* energy;
  int ecap;
  double* probes;
  int pcap;
  double* partials;
  StepState* st;
  double dt, eps0, mu0;
  int nblocks;
  int t0, t1;  // tile range of this launch
  int poff;    // first partial-sum slot of this launch
  int hpoff;   // E launches: first slot of the H launch over the same tiles
               // (its partial joins the E workgroup's), else -1
  const struct TfDesc* tf;  // total-field / scattered-field injection, or null
};

// Field pools of step n: the one it reads (the state E^n, H^{n-1/2}) and
// the one it writes (E^{n+1}, H^{n+1/2}).
__device__ __forceinline__ void* pool_in(const KArgs& a, long long n) { return (n & 1) ? a.pool2 : a.pool; }
__device__ __forceinline__ void* pool_out(const KArgs& a, long long n) { return (n & 1) ? a.pool : a.pool2; }


// Near box of a block for local time stepping: node index ranges [lo, hi]
// per axis (inclusive); on = 0: no node of the block is near a refined block.
struct LtsBox {
  int lo[3], hi[3];
  int on, refined;
};

// ------------------------------------------------ E-node material helpers
// (the adjoint's gradient and the local time stepping's energy)
// Sum S of eps_r over the four clamped cells around E node (i, j, k) of
// component c (Ex: {ci0} x {cj0, cj1} x {ck0, ck1}; Ey: {ci0, ci1} x {cj0} x
// {ck0, ck1}; Ez: {ci0, ci1} x {cj0, cj1} x {ck0}, ci0 = clamp(i-1),
// ci1 = clamp(i), ...), and the four cells (repeated where clamped).
struct NodeCells {
  double S;
  int cell[4];  // block-local cell indices ci + nx (cj + ny ck)
};

template <typename T>
__device__ __forceinline__ const T* cells_of_block(const void* mat_eps, const DevBlock& B) {
  return mat_eps ? (const T*)mat_eps + B.coff : nullptr;
}

// Norm weight w_E of E node (i, j, k) of component c: the product of the 1D
// weights (Appendix P+, P-) with h.  The full geometric weight (not w / h^3)
// keeps the adjoint variables of blocks of different mesh sizes consistent.
__device__ __forceinline__ double e_weight(const DevBlock& B, int c, int i, int j, int k) {
  const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
  const double wx = c == 0 ? wm1(nx, i) : wp1(nx, i);
  const double wy = c == 1 ? wm1(ny, j) : wp1(ny, j);
  const double wz = c == 2 ? wm1(nz, k) : wp1(nz, k);
  return (wx * B.h[0]) * (wy * B.h[1]) * (wz * B.h[2]);
}

// dte0x4 / S: the E-update coefficient Cb of a lossless node (double).
__device__ __forceinline__ double node_cb(const DevBlock& B, double S) { return B.dte0x4 / S; }

template <typename T>
__device__ inline NodeCells node_cells_t(const DevBlock& B, const void* mat_eps, int c, int i, int j, int k) {
  const T* cv = cells_of_block<T>(mat_eps, B);
  const bool has_eps = (B.mat & MAT_EPS) && cv;
  const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
  NodeCells r;
  const int ci0 = clampi(i - 1, 0, nx - 1), ci1 = clampi(i, 0, nx - 1);
  const int cj0 = clampi(j - 1, 0, ny - 1), cj1 = clampi(j, 0, ny - 1);
  const int ck0 = clampi(k - 1, 0, nz - 1), ck1 = clampi(k, 0, nz - 1);
  int q = 0;
  r.S = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      int ci, cj, ck;
      if (c == 0) { ci = ci0; cj = a ? cj1 : cj0; ck = b ? ck1 : ck0; }
      else if (c == 1) { ci = a ? ci1 : ci0; cj = cj0; ck = b ? ck1 : ck0; }
      else { ci = a ? ci1 : ci0; cj = b ? cj1 : cj0; ck = ck0; }
      const int cell = ci + nx * (cj + ny * ck);
      r.cell[q++] = cell;
      r.S += has_eps ? (double)cv[cell] : B.eps_r0;
    }
  return r;
}


}  // namespace sbp
