// Leapfrog step kernels of the 3D SBP-SAT FDTD method for gfx950.
//
// Memory-bound staggered stencil, one launch per half step over every node
// of every block.  A tile is a run of consecutive nodes of the flattened
// (i fastest) xy node plane of one block; each thread owns one (i, j) node
// column and marches through the tile's z planes, so the z-neighbour of the
// previous plane stays in registers and every wave reads 64 contiguous
// values per array.  Interior rows are the two-point Yee difference (Section
// II-A: the interior nodes are Yee's); rows within two (D+) or three (D-)
// nodes of a block face take the Appendix closure rows with the SAT row
// changes folded in (PEC in the H update, PMC / absorbing in the E update,
// interface rows adding the gathered neighbour value): per lane for x, per
// thread for y, per plane (wave-uniform) for z.  The field update runs in
// the field precision; the energy sums, the interface interpolation and the
// interface penalty (the neighbour's value joining a boundary row) are
// formed in fp64, the interface row being narrowed once.  Every node update
// is a pure function of the previous fields, so the results do not depend on
// the tile shape or on how tiles map to workgroups.
//
// The tile list is walked XCD-aware (TileIter): groups of consecutive tiles
// go to one XCD, so the y-neighbour rows a tile re-reads were mostly fetched
// into the same L2 by the tile before it.
//
// The discrete energy W^n (E16 with the leapfrog pairing of H) is summed in
// fp64 per workgroup; the E workgroup of a tile adds the H partial of the
// same tile to its own, and k_finish sums the partials in a fixed order.

#include "plan.h"

namespace sbp {

constexpr int kXcds = 8;  // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kGroup = 8;  // tiles per XCD group in the dispatch-order tile walk


// Workgroup sum of `v`, stored to partials[poff + blockIdx.x]; the launch's
// total is formed later by k_finish, in a fixed order (deterministic).
__device__ void store_partial(double v, const KArgs& a) {
  __shared__ double red[16];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    if (a.hpoff >= 0) s += a.partials[a.hpoff + blockIdx.x];  // the H partial of the same tile
    a.partials[a.poff + blockIdx.x] = s;
  }
}

__device__ __forceinline__ double waveform(const Source& s, double t) {
  const double d = t - s.t0;
  const double g = exp(-4.0 * M_PI * d * d / (s.tw * s.tw));
  return s.wave == 1 ? sin(2.0 * M_PI * s.f0 * t) * g : g;
}

// Current density of every source at (n+1/2) dt, n the step index.
__device__ __forceinline__ void eval_sources(const KArgs& a, long long n) {
  const double t = ((double)n + 0.5) * a.dt;
  for (int p = threadIdx.x; p < a.nsrc; p += blockDim.x) a.srcval[p] = a.src[p].amp * waveform(a.src[p], t);
}

// Source values of the current step (before the first step of a call, or
// after the state was replaced).
__global__ __launch_bounds__(256) void k_sources(KArgs a) { eval_sources(a, a.st->step); }

// End of step n: steps the TF/SF incident line (if any), sums partials[p0
// .. nparts) (one workgroup, fixed order) into energy ring slot n (W^n),
// flags a non-finite energy, advances the step index and evaluates the
// source values of step n+1.
__global__ __launch_bounds__(1024) void k_finish(KArgs a, int p0, int nparts) {
  __shared__ double red[16];
  const long long n = a.st->step;  // read first: the source values below need it, not the partials
  if (a.tf) {
    // the TF/SF incident line, stepped one half step ahead of the 3D fields:
    // E^{n+1} with the source value of step n (at (n + 1/2) dt), then
    // H^{n+3/2}, which the E update of step n+1 reads (the H update of step
    // n+1 reads E^{n+1}).  One-dimensional leapfrog along the propagation
    // axis with the interior difference, PEC ends.
    const TfDesc& tf = *a.tf;
    double* e1 = tf.e1;
    double* h1 = tf.h1;
    const int len = tf.len;
    const double ce = tf.ce, ch = tf.ch, se = a.dt / a.eps0 * a.srcval[tf.sidx];
    for (int i = 1 + threadIdx.x; i < len; i += blockDim.x)
      e1[i] += ce * (h1[i] - h1[i - 1]) + (i == tf.src ? se : 0.0);
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += blockDim.x) h1[i] += ch * (e1[i + 1] - e1[i]);
    __syncthreads();  // the source values of step n are read before they are replaced
  }
  // eight independent running sums per thread keep eight loads in flight
  // (the partials come from other XCDs' caches); fixed order for a given
  // nparts and block size
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int nb = blockDim.x;
  int p = p0 + threadIdx.x;
  for (; p + 7 * nb < nparts; p += 8 * nb)
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += a.partials[p + u * nb];
  for (; p < nparts; p += nb) acc[0] += a.partials[p];
  eval_sources(a, n + 1);  // its arithmetic overlaps the partials' loads
  double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  s = wave_sum(s);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0) red[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < nw; ++w) tot += red[w];
    a.energy[(int)(n % a.ecap)] = tot;
    if (!isfinite(tot)) a.st->flags |= 1;
    a.st->step = n + 1;
  }
}

// Walks the tile list.  order 0: a workgroup per tile takes the tiles in
// (grouped) dispatch order, so the workgroups resident at any moment stream
// through neighbouring addresses (faster for state larger than the
// last-level cache).
// order 1, or a persistent grid (fewer workgroups than tiles): the workgroups
// on one XCD (workgroup g sits on XCD g % 8) take a contiguous range of
// tiles, which keeps neighbouring planes in that XCD's L2 (faster for
// cache-resident state).  The host rounds the grid up to a multiple of 8;
// surplus workgroups only join the energy reduction.
struct TileIter {
  int t, stop, stride;
  __device__ TileIter(int ntiles, int order) {
    const int g = blockIdx.x, G = gridDim.x;
    if ((order == 1 || G < ntiles) && G % kXcds == 0) {
      const int per = (ntiles + kXcds - 1) / kXcds;
      const int x = g % kXcds;
      t = x * per + g / kXcds;
      stop = min((x + 1) * per, ntiles);
      stride = G / kXcds;
    } else {
      // groups of kGroup consecutive tiles (about four node rows at 128
      // threads) go to one XCD, consecutive groups to the next XCDs: the
      // workgroups resident at a time still cover neighbouring addresses,
      // and the row behind a tile (its y neighbours) is mostly in the same
      // XCD's L2.  The last partial round of groups keeps dispatch order.
      const int w = g / kXcds, x = g % kXcds, full = (G / kXcds) / kGroup * kGroup;
      t = w < full ? ((w / kGroup) * kXcds + x) * kGroup + w % kGroup : g;
      stop = ntiles;
      stride = G;
    }
  }
  __device__ bool next(int& out) {
    if (t >= stop) return false;
    out = t;
    t += stride;
    return true;
  }
};

// Material coefficients q / d (Cb, Db and the loss factors; d >= 1 times
// a positive constant): fp32 multiplies by the hardware reciprocal (within
// 1 ulp of 1/d, so within 2 ulp of the quotient), fp64 divides.
template <typename T>
__device__ __forceinline__ T quot(T q, T d) {
  if constexpr (sizeof(T) == 4) return q * __builtin_amdgcn_rcpf(d);
  else return q / d;
}

// ------------------------------------------------------------- rows
// One row of D+ or D- along an axis at node index r, coefficients in the
// field precision: interior rows are flagged (two-point difference), closure
// rows read three consecutive nodes r+s .. r+s+2 (Appendix rows with the
// Section III SAT row changes), plus cn times the gathered neighbour value on
// interface faces.  Rows outside the operator's range (components that do
// not exist there) are zero.
template <typename T>
struct TRow {
  int s, nbr, in;
  T c0, c1, c2, cn;
};

template <typename T, typename DB>
__device__ __forceinline__ TRow<T> row_of(const DB& B, int axis, int r, bool minus) {
  TRow<T> R;
  const int n = B.n[axis];
  R.nbr = 0;
  R.cn = T(0);
  R.in = minus ? (r >= 3 && r <= n - 2) : (r >= 2 && r <= n - 2);
  if (R.in) {
    R.s = minus ? -1 : 0;
    R.c0 = -(T)B.ih[axis];
    R.c1 = (T)B.ih[axis];
    R.c2 = T(0);
  } else if (!minus && r > n) {  // no D+ row: the E component does not exist here
    R.s = -2;
    R.c0 = R.c1 = R.c2 = T(0);
  } else {
    const auto& X = minus ? B.dm[axis][r < 3 ? r : r - (n - 1) + 3] : B.dp[axis][r < 2 ? r : r - (n - 1) + 2];
    R.s = X.s;
    R.c0 = (T)X.c[0];
    R.c1 = (T)X.c[1];
    R.c2 = (T)X.c[2];
    R.nbr = X.nbr;
    R.cn = (T)X.cn;
  }
  return R;
}

// The x closure rows from values the march loads with the plane: besides
// the node (d = 0) and its interior partner (d = -1 for D-, +1 for D+), each
// boundary row reads at most one more node, at offset h_xd / e_xd (0: none);
// taps with a zero coefficient read nothing.  Loaded in place, these values
// would wait behind the next plane's loads (vector memory loads complete in
// order).
__device__ __forceinline__ int h_xd(int i, int n) {  // D- rows 0, 2, n-1, n+1
  return (i == 0 || i == n - 1) ? 1 : ((i == 2 || i == n + 1) ? -2 : 0);
}
__device__ __forceinline__ int e_xd(int i, int n) {  // D+ rows 0, 1, n-1, n
  return (i == 0 || i == n - 1) ? 2 : ((i == 1 || i == n) ? -1 : 0);
}

template <typename T>
__device__ __forceinline__ T xrow(const TRow<T>& R, T u0, T un, int dn, T ux, int xd) {
  auto pick = [&](int d) { return d == 0 ? u0 : (d == dn ? un : (d == xd ? ux : T(0))); };
  return R.c0 * pick(R.s) + R.c1 * pick(R.s + 1) + R.c2 * pick(R.s + 2);
}

// Interface row: the own-value part r (field precision) plus the gathered
// neighbour value f (fp64) times the row's neighbour coefficient, which is
// -1/h on a low face and +1/h on a high face.  The penalty is added in fp64
// and the row narrowed once.
template <typename T>
__device__ __forceinline__ T pen(T r, T cn, double ih, double f) {
  return (T)((double)r + (cn > T(0) ? ih : -ih) * f);
}

// Closure row applied to u along stride st at node offset o; on an
// interface row the gathered neighbour value a.face[fo] joins it (ih: 1/h
// of the row's axis in fp64).
template <typename T, bool IFACE>
__device__ __forceinline__ T drow(const KArgs& a, const T* __restrict__ u, long long o, long long st,
                                  const TRow<T>& R, long long fo, double ih) {
  const T* p = u + o + (long long)R.s * st;
  T v = R.c0 * p[0] + R.c1 * p[st] + R.c2 * p[2 * st];
  if constexpr (IFACE) {
    if (R.nbr) v = pen<T>(v, R.cn, ih, a.face[fo]);
  }
  return v;
}

// Probe samples of node (i, j, k): probes of the given field on that node
// take the new values (only for tiles flagged as holding a probe).
template <typename T>
__device__ __forceinline__ void take_probes(const KArgs& a, const DevBlock& B, int i, int j, int k, bool h_field,
                                            long long nstep, T v0, T v1, T v2) {
  for (int p = 0; p < B.nprb; ++p) {
    const Probe& P = a.prb[B.prb0 + p];
    if ((P.comp >= HX) == h_field && P.i == i && P.j == j && P.k == k) {
      const int c = P.comp % 3;
      a.probes[(long long)(B.prb0 + p) * a.pcap + nstep % a.pcap] = (double)(c == 0 ? v0 : (c == 1 ? v1 : v2));
    }
  }
}

// Current density of the block's sources on node (i, j, k) (tiles flagged
// as holding a source), from the values the finish kernel evaluated.
template <typename T>
__device__ __forceinline__ void source_terms(const KArgs& a, const DevBlock& B, int i, int j, int k, T& jx, T& jy,
                                             T& jz) {
  for (int p = 0; p < B.nsrc; ++p) {
    const Source& S = a.src[B.src0 + p];
    if (S.i == i && S.j == j && S.k == k) {
      const T v = (T)a.srcval[B.src0 + p];
      jx += S.comp == EX ? v : T(0);
      jy += S.comp == EY ? v : T(0);
      jz += S.comp == EZ ? v : T(0);
    }
  }
}

// Read-only tables (block descriptors, tile list) are read through the
// constant address space so that wave-uniform reads become scalar loads.
#define SBP_CONST __attribute__((address_space(4)))
template <typename X>
__device__ __forceinline__ const SBP_CONST X* as_const(const X* p) {
  return (const SBP_CONST X*)p;
}

// Face-buffer offsets of a node column's x- and y-face interface rows: the
// buffer of face f holds, per slot (is_h * 2 + tangential component), the
// face's nodes in its own (x fastest) order: (j, k) on x faces, (i, k) on y
// faces, (i, j) on z faces.  `lo` splits the column's rows between the low
// and the high face.
struct FaceCol {
  long long x, y;
};
__device__ __forceinline__ FaceCol face_col(const SBP_CONST DevBlock& Bc, int i, int j, int lo) {
  return FaceCol{(i < lo ? Bc.fboff[0] : Bc.fboff[1]) + j, (j < lo ? Bc.fboff[2] : Bc.fboff[3]) + i};
}

// Absorbing layers (convolutional PML): profile value q (0: b, 1: c,
// 2: 1/kappa) of axis `axis`, grid g (0: "+", 1: "-") at node index idx.
template <typename T>
__device__ __forceinline__ T pml_at(const KArgs& a, const SBP_CONST DevBlock& Bc, int axis, int g, int q, int idx) {
  return ((const T*)a.pml_prof)[Bc.pml_off + (long long)((axis * 2 + g) * 3 + q) * Bc.pml_stride + idx];
}
// A node column's x and y profile values (hoisted out of the march).
template <typename T>
struct PmlCol {
  T bx, cx, kx, by, cy, ky;
};
template <typename T>
__device__ __forceinline__ PmlCol<T> pml_col(const KArgs& a, const SBP_CONST DevBlock& Bc, int g, int i, int j) {
  return PmlCol<T>{pml_at<T>(a, Bc, 0, g, 0, i), pml_at<T>(a, Bc, 0, g, 1, i), pml_at<T>(a, Bc, 0, g, 2, i),
                   pml_at<T>(a, Bc, 1, g, 0, j), pml_at<T>(a, Bc, 1, g, 1, j), pml_at<T>(a, Bc, 1, g, 2, j)};
}
// ------------------------------------------------------------- TF/SF
// Membership of a node index along one axis in the total-field box
// [lo h, hi h]: "+" nodes lo..hi, "-" nodes lo+1..hi.
__device__ __forceinline__ bool tf_in(bool plus, int idx, int lo, int hi) {
  return plus ? (idx >= lo && idx <= hi) : (idx >= lo + 1 && idx <= hi);
}

// Component v (0, 1, 2) of (i, j, k), without a local array (a dynamic
// index into one would go through scratch memory).
__device__ __forceinline__ int sel3(int v, int i, int j, int k) { return v == 0 ? i : (v == 1 ? j : k); }

// Whether node (i, j, k) can take a correction: all indices within one of
// the box and one of them on its edge (lo - 1, lo, hi or hi + 1).
__device__ __forceinline__ bool tf_near(const SBP_CONST TfDesc& tf, int i, int j, int k) {
  bool in = true, edge = false;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int x = b == 0 ? i : (b == 1 ? j : k), lo = tf.lo[b], hi = tf.hi[b];
    in = in && x >= lo - 1 && x <= hi + 1;
    edge = edge || x <= lo || x >= hi;
  }
  return in && edge;
}

// The corrections of a node across the TF/SF surface.  Two curl terms
// difference the incident component (on the H side: the H components other
// than the incident E one; on the E side likewise).  A term's difference
// along `ax` (two-point: the box lies in the interior) couples the node
// (grid type "-" along ax for H, "+" for E; index pa) to the source
// component's nodes q of the other grid type (H: pa-1, pa; E: pa, pa+1).
// Where p and q lie on opposite sides of the surface (at most one q per term,
// the box being at least a cell thick), the incident value of q joins the
// node's update, + in the total region and - in the scattered one (the
// neighbour's value taken in the node's own convention), times the
// difference's coefficient -1/h (first q) or +1/h (second q).  Along the
// other two axes p and q share index and grid type, so they must lie inside
// the box there.
//
// tf_gather finds, per term, the sign of the correction (0: none) and loads
// the incident value.  The E kernel gathers one plane ahead, with the field
// values of that plane, so that these loads do not wait behind the next
// plane's (vector memory loads complete in order).
struct TfPre {
  double v[2];
  int s[2];
};

template <bool E_SIDE>
__device__ __forceinline__ void tf_gather(const KArgs& a, int i, int j, int k, TfPre& p) {
  p.v[0] = p.v[1] = 0.0;
  p.s[0] = p.s[1] = 0;
  const SBP_CONST TfDesc& tf = *as_const(a.tf);
  if (!tf_near(tf, i, j, k)) return;
  const int pr = tf.axis, margin = tf.margin;
  const int pprop = sel3(pr, i, j, k);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int c = E_SIDE ? tf.e_comp[t] : tf.h_comp[t];
    const int ax = E_SIDE ? tf.e_ax[t] : tf.h_ax[t];
    const int o = 3 - c - ax;
    const double sg = E_SIDE ? tf.e_sg[t] : tf.h_sg[t];
    // H_c is "+" along c and "-" along o; E_c is "-" along c and "+" along o
    const bool other = tf_in(!E_SIDE, sel3(c, i, j, k), tf.lo[c], tf.hi[c]) &&
                       tf_in(E_SIDE, sel3(o, i, j, k), tf.lo[o], tf.hi[o]);
    if (!other) continue;
    const int pa = sel3(ax, i, j, k), lo = tf.lo[ax], hi = tf.hi[ax];
    const bool pin = tf_in(E_SIDE, pa, lo, hi);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int qa = pa + (E_SIDE ? q : q - 1);
      if (tf_in(!E_SIDE, qa, lo, hi) == pin) continue;
      const int ip = ax == pr ? qa : pprop;  // the source node's index along the propagation
      p.v[t] = E_SIDE ? tf.h1[ip - 1 + margin] : tf.e1[ip + margin];
      p.s[t] = ((pin ? sg : -sg) > 0.0) == (q == 1) ? 1 : -1;
    }
  }
}

// The same corrections, gathered and combined in one go (the H kernel).
template <bool E_SIDE, typename T>
__device__ __forceinline__ void tf_terms(const KArgs& a, const SBP_CONST DevBlock& Bc, int i, int j, int k, T& cx,
                                         T& cy, T& cz) {
  const SBP_CONST TfDesc& tf = *as_const(a.tf);
  const int pr = tf.axis, margin = tf.margin;
  const int pprop = sel3(pr, i, j, k);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int c = E_SIDE ? tf.e_comp[t] : tf.h_comp[t];
    const int ax = E_SIDE ? tf.e_ax[t] : tf.h_ax[t];
    const int o = 3 - c - ax;
    const double sg = E_SIDE ? tf.e_sg[t] : tf.h_sg[t], ih = Bc.ih[ax];
    // H_c is "+" along c and "-" along o; E_c is "-" along c and "+" along o
    const bool other = tf_in(!E_SIDE, sel3(c, i, j, k), tf.lo[c], tf.hi[c]) &&
                       tf_in(E_SIDE, sel3(o, i, j, k), tf.lo[o], tf.hi[o]);
    if (!other) continue;
    const int pa = sel3(ax, i, j, k), lo = tf.lo[ax], hi = tf.hi[ax];
    const bool pin = tf_in(E_SIDE, pa, lo, hi);
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int qa = pa + (E_SIDE ? q : q - 1);
      if (tf_in(!E_SIDE, qa, lo, hi) == pin) continue;
      const int ip = ax == pr ? qa : pprop;  // the source node's index along the propagation
      const double v = E_SIDE ? tf.h1[ip - 1 + margin] : tf.e1[ip + margin];
      acc += (q ? ih : -ih) * v;
    }
    const T d = (T)((pin ? sg : -sg) * acc);
    cx += c == 0 ? d : T(0);
    cy += c == 1 ? d : T(0);
    cz += c == 2 ? d : T(0);
  }
}

template <bool E_SIDE, typename T>
__device__ __forceinline__ void tf_combine(const KArgs& a, const SBP_CONST DevBlock& Bc, const TfPre& p, T& cx, T& cy,
                                           T& cz) {
  const SBP_CONST TfDesc& tf = *as_const(a.tf);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int c = E_SIDE ? tf.e_comp[t] : tf.h_comp[t];
    const int ax = E_SIDE ? tf.e_ax[t] : tf.h_ax[t];
    const T d = (T)((double)p.s[t] * Bc.ih[ax] * p.v[t]);
    cx += c == 0 ? d : T(0);
    cy += c == 1 ? d : T(0);
    cz += c == 2 ? d : T(0);
  }
}

// Stretched difference inside a layer: psi <- b psi + c d, d <- d / kappa +
// psi; `old` is psi as loaded with the plane's field values.
template <typename T>
__device__ __forceinline__ void stretch(T& d, T b, T c, T ik, T* psi, T old) {
  const T p = b * old + c * d;
  *psi = p;
  d = d * ik + p;
}

// z profile value q of grid g at plane k (wave-uniform: a scalar load).
template <typename T>
__device__ __forceinline__ T pml_z(const KArgs& a, const SBP_CONST DevBlock& Bc, int g, int q, int k) {
  return as_const((const T*)a.pml_prof)[Bc.pml_off + (long long)((2 * 2 + g) * 3 + q) * Bc.pml_stride + k];
}

// The recursion variables a node of plane k updates (the kernels load them
// one plane ahead, with the field values, so that they do not wait behind
// the next plane's loads).  H slots 0-5: (Hx,z) (Hx,y) (Hy,x) (Hy,z) (Hz,y)
// (Hz,x); E slots 6-11: (Ex,y) (Ex,z) (Ey,z) (Ey,x) (Ez,x) (Ez,y).
template <typename T, bool E_SIDE>
__device__ __forceinline__ void psi_load(const KArgs& a, const SBP_CONST DevBlock& Bc, const PmlCol<T>& pc, int k,
                                         long long o, T (&v)[6]) {
  const T* ps = (const T*)a.psi + Bc.psi_off + (E_SIDE ? 6 * Bc.csz : 0) + o;
  const long long cs = Bc.csz;
  const int g = E_SIDE ? 0 : 1;
  const bool zl = (!E_SIDE || k <= Bc.n[2]) && (pml_z<T>(a, Bc, g, 1, k) != T(0) || pml_z<T>(a, Bc, g, 2, k) != T(1));
  const int z0 = E_SIDE ? 1 : 0, z1 = E_SIDE ? 2 : 3;  // slots of the z terms
  const int y0 = E_SIDE ? 0 : 1, y1 = E_SIDE ? 5 : 4;  // y terms
  const int x0 = E_SIDE ? 3 : 2, x1 = E_SIDE ? 4 : 5;  // x terms
  if (zl) {
    v[z0] = ps[z0 * cs];
    v[z1] = ps[z1 * cs];
  }
  if (pc.cy != T(0) || pc.ky != T(1)) {
    v[y0] = ps[y0 * cs];
    v[y1] = ps[y1 * cs];
  }
  if (pc.cx != T(0) || pc.kx != T(1)) {
    v[x0] = ps[x0 * cs];
    v[x1] = ps[x1 * cs];
  }
}

// Element `idx` of a component array addressed as the (wave-uniform) array
// base plus a 32-bit byte offset, so that an access costs one vector offset
// instead of a 64-bit address.  Component arrays stay below 4 GiB (checked
// when a block is added).
template <typename T>
__device__ __forceinline__ T ld32(const T* base, unsigned idx) {
  return *(const T*)((const char*)base + (size_t)(idx * (unsigned)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st32(T* base, unsigned idx, T v) {
  *(T*)((char*)base + (size_t)(idx * (unsigned)sizeof(T))) = v;
}

// Per-tile copy of the block constants the node updates use (registers;
// the closure tables stay in the descriptor, read by boundary rows only).
template <typename T>
struct BC {
  int nx, ny, nz, mat, abc;
  long long sx, sxy;
  T ihx, ihy, ihz;
  T db_u, dtm0x2, mu_r0;               // H update
  T cb_u, dte0x4, hdte0, eps_r0, sig0;  // E update
  long long coff;
  __device__ explicit BC(const SBP_CONST DevBlock& B) {
    nx = B.n[0]; ny = B.n[1]; nz = B.n[2]; mat = B.mat; abc = B.abc_mask;
    sx = B.sx; sxy = B.sxy; coff = B.coff;
    ihx = (T)B.ih[0]; ihy = (T)B.ih[1]; ihz = (T)B.ih[2];
    db_u = (T)B.db_u; dtm0x2 = (T)B.dtm0x2; mu_r0 = (T)B.mu_r0;
    cb_u = (T)B.cb_u; dte0x4 = (T)B.dte0x4; hdte0 = (T)B.hdte0; eps_r0 = (T)B.eps_r0; sig0 = (T)B.sig0;
  }
};

// Norm weights / h^3 of a node column's three components without the z
// factor (which the plane supplies), zero for components that do not exist
// in the column.
template <typename T>
struct W3 {
  T x, y, z;
};
template <typename T>
__device__ __forceinline__ W3<T> h_col_weights(int nx, int ny, int i, int j) {
  return W3<T>{i <= nx ? (T)(wp1(nx, i) * wm1(ny, j)) : T(0), j <= ny ? (T)(wm1(nx, i) * wp1(ny, j)) : T(0),
               (T)(wm1(nx, i) * wm1(ny, j))};
}
template <typename T>
__device__ __forceinline__ W3<T> e_col_weights(int nx, int ny, int i, int j) {
  return W3<T>{j <= ny ? (T)(wm1(nx, i) * wp1(ny, j)) : T(0), i <= nx ? (T)(wp1(nx, i) * wm1(ny, j)) : T(0),
               (i <= nx && j <= ny) ? (T)(wp1(nx, i) * wp1(ny, j)) : T(0)};
}

// ------------------------------------------------------------- H update
// Field values one H node update reads at interior rows: E and H at the
// node, E one node back along y and x (offsets kept inside the component
// box on the first row / column) and Ex, Ey one plane back.  A thread walks
// a column of planes: the plane-back values are the previous plane's centre
// values, carried in registers, and the next plane is loaded before the
// current one is computed.
template <typename T>
struct HIn {
  T ex, ey, ez, hx, hy, hz;
  T ey_z, ex_z, ez_y, ex_y, ez_x, ey_x;
  T ez_xx, ey_xx;  // x closure rows: the value beyond the interior pair (h_xd)
  double ez_f, ey_f;  // interface x rows: the neighbour's face values (fp64)
  T ez_yy, ex_yy;     // y rows of interface blocks: likewise
  double ez_fy, ex_fy;
  T ey_zz, ex_zz;     // z rows of interface blocks: likewise
  double ey_fz, ex_fz;
  T psi[6];  // absorbing layers: the node's recursion variables (slots 0-5)
};

template <typename T>
__device__ __forceinline__ void h_load(HIn<T>& v, const BC<T>& c, const T* __restrict__ Ex,
                                       const T* __restrict__ Ey, const T* __restrict__ Ez,
                                       const T* __restrict__ Hx, const T* __restrict__ Hy,
                                       const T* __restrict__ Hz, int i, int j, long long o) {
  const unsigned u = (unsigned)o, uy = u - (j > 0 ? (unsigned)c.sx : 0u), ux = u - (i > 0 ? 1u : 0u);
  v.ex = ld32(Ex, u);
  v.ey = ld32(Ey, u);
  v.ez = ld32(Ez, u);
  v.hx = ld32(Hx, u);
  v.hy = ld32(Hy, u);
  v.hz = ld32(Hz, u);
  v.ez_y = ld32(Ez, uy);
  v.ex_y = ld32(Ex, uy);
  v.ez_x = ld32(Ez, ux);
  v.ey_x = ld32(Ey, ux);
  const int xd = h_xd(i, c.nx);
  if (xd != 0) {
    v.ez_xx = ld32(Ez, u + (unsigned)xd);
    v.ey_xx = ld32(Ey, u + (unsigned)xd);
  }
}

// Interface x rows of plane k: the neighbour's face values (face buffer,
// fp64), the Ez and Ey slots of the x face.
template <typename T>
__device__ __forceinline__ void h_face(const KArgs& a, const BC<T>& c, const FaceCol& fc, int k, HIn<T>& v) {
  const long long by = c.ny + 2, bz = c.nz + 2, fo = fc.x + by * k;
  v.ez_f = a.face[fo + by * bz];
  v.ey_f = a.face[fo];
}

// The z rows of an interface block at plane k (wave-uniform: only the planes
// next to the z faces), with the Ey and Ex slots of the z face.
template <typename T>
__device__ __forceinline__ void h_zrow(const KArgs& a, const BC<T>& c, const SBP_CONST DevBlock& Bc,
                                       const T* __restrict__ Ey, const T* __restrict__ Ex, int i, int j, int k,
                                       long long o, HIn<T>& v) {
  if (k >= 3 && k <= c.nz - 2) return;
  const int zd = h_xd(k, c.nz);
  if (zd != 0) {
    const unsigned u = (unsigned)o + (unsigned)(zd * (int)c.sxy);
    v.ey_zz = ld32(Ey, u);
    v.ex_zz = ld32(Ex, u);
  }
  if (row_of<T>(Bc, 2, k, true).nbr) {
    const long long bx = c.nx + 2, by = c.ny + 2, fo = Bc.fboff[k < 3 ? 4 : 5] + i + bx * j;
    v.ey_fz = a.face[fo + bx * by];
    v.ex_fz = a.face[fo];
  }
}

// The y rows of an interface block at plane k from loads issued with the
// plane: the node beyond the interior pair, and on an interface face the
// neighbour's face values (Ez and Ex slots of the y face).  Only interface
// blocks take these: they are small, so their boundary rows are a larger
// share of the waves, and the plain kernels keep their registers.
template <typename T>
__device__ __forceinline__ void h_yrow(const KArgs& a, const BC<T>& c, const FaceCol& fc, const TRow<T>& ry,
                                       const T* __restrict__ Ez, const T* __restrict__ Ex, int j, int k,
                                       long long o, HIn<T>& v) {
  const int yd = h_xd(j, c.ny);
  if (yd != 0) {
    const unsigned u = (unsigned)o + (unsigned)(yd * (int)c.sx);
    v.ez_yy = ld32(Ez, u);
    v.ex_yy = ld32(Ex, u);
  }
  if (ry.nbr) {
    const long long bx = c.nx + 2, bz = c.nz + 2, fo = fc.y + bx * k;
    v.ez_fy = a.face[fo + bx * bz];
    v.ex_fy = a.face[fo];
  }
}

// H^{n+1/2} = H^{n-1/2} + dt/mu (E10-E12) at node (i, j, k), all valid H
// components, with the closure / PEC / interface rows replacing the interior
// differences on the boundary rows.  Returns the node's
// (w/h^3) mu_r H^{n+1/2} H^{n-1/2}.
template <typename T, bool GEN, bool IFACE, bool PML, bool TF = false>
__device__ __forceinline__ T h_node(const KArgs& a, const SBP_CONST DevBlock& Bc,
                                    const TRow<T>& rx, const TRow<T>& ry, const W3<T>& lw, const BC<T>& c,
                                    const HIn<T>& v,
                                    const T* __restrict__ Ex, const T* __restrict__ Ey,
                                    const T* __restrict__ Ez, T* __restrict__ Hx, T* __restrict__ Hy,
                                    T* __restrict__ Hz, const T* __restrict__ M, const FaceCol& fc,
                                    const PmlCol<T>& pc, T tcx, T tcy, T tcz, int i, int j, int k, long long o,
                                    bool store, T& onx, T& ony, T& onz) {
  const int nx = c.nx, ny = c.ny, nz = c.nz;
  const long long sx = c.sx, sxy = c.sxy;
  const T ihx = c.ihx, ihy = c.ihy, ihz = c.ihz;
  const T hx = v.hx, hy = v.hy, hz = v.hz;
  const bool xin = i >= 3 && i <= nx - 2, yin = j >= 3 && j <= ny - 2, zin = k >= 3 && k <= nz - 2;
  T dzEy = (v.ey - v.ey_z) * ihz, dzEx = (v.ex - v.ex_z) * ihz;
  T dyEz = (v.ez - v.ez_y) * ihy, dyEx = (v.ex - v.ex_y) * ihy;
  T dxEz = (v.ez - v.ez_x) * ihx, dxEy = (v.ey - v.ey_x) * ihx;
  // face-buffer slots of tangential E: 0 and 1 (ascending tangential axis)
  const long long bx = nx + 2, by = ny + 2, bz = nz + 2;
  if (!zin) {
    const TRow<T> rz = row_of<T>(Bc, 2, k, true);
    if constexpr (IFACE && sizeof(T) == 4) {  // (fp64: registers would spill)
      // interior pair: E at k (v.ey) and k-1 (v.ey_z)
      const int zd = h_xd(k, nz);
      dzEy = xrow<T>(rz, v.ey, v.ey_z, -1, v.ey_zz, zd);
      dzEx = xrow<T>(rz, v.ex, v.ex_z, -1, v.ex_zz, zd);
      if (rz.nbr) {
        dzEy = pen<T>(dzEy, rz.cn, Bc.ih[2], v.ey_fz);
        dzEx = pen<T>(dzEx, rz.cn, Bc.ih[2], v.ex_fz);
      }
    } else {
      const long long fo = Bc.fboff[k < 3 ? 4 : 5] + i + bx * j;
      dzEy = drow<T, IFACE>(a, Ey, o, sxy, rz, fo + bx * by, Bc.ih[2]);
      dzEx = drow<T, IFACE>(a, Ex, o, sxy, rz, fo, Bc.ih[2]);
    }
  }
  if (!yin) {
    if constexpr (IFACE) {
      const int yd = h_xd(j, ny);
      dyEz = xrow<T>(ry, v.ez, v.ez_y, -1, v.ez_yy, yd);
      dyEx = xrow<T>(ry, v.ex, v.ex_y, -1, v.ex_yy, yd);
      if (ry.nbr) {
        dyEz = pen<T>(dyEz, ry.cn, Bc.ih[1], v.ez_fy);
        dyEx = pen<T>(dyEx, ry.cn, Bc.ih[1], v.ex_fy);
      }
    } else {
      const long long fo = fc.y + bx * k;
      dyEz = drow<T, IFACE>(a, Ez, o, sx, ry, fo + bx * bz, Bc.ih[1]);
      dyEx = drow<T, IFACE>(a, Ex, o, sx, ry, fo, Bc.ih[1]);
    }
  }
  if (!xin) {
    const int xd = h_xd(i, nx);
    dxEz = xrow<T>(rx, v.ez, v.ez_x, -1, v.ez_xx, xd);
    dxEy = xrow<T>(rx, v.ey, v.ey_x, -1, v.ey_xx, xd);
    if (IFACE && rx.nbr) {
      dxEz = pen<T>(dxEz, rx.cn, Bc.ih[0], v.ez_f);
      dxEy = pen<T>(dxEy, rx.cn, Bc.ih[0], v.ey_f);
    }
  }
  if constexpr (PML) {  // absorbing layers: H terms sit on the "-" grid of their axis
    T* ps = (T*)a.psi + Bc.psi_off + o;  // slots 0-5: (Hx,z) (Hx,y) (Hy,x) (Hy,z) (Hz,y) (Hz,x)
    const long long cs = Bc.csz;
    const T bzp = pml_z<T>(a, Bc, 1, 0, k), czp = pml_z<T>(a, Bc, 1, 1, k), kzp = pml_z<T>(a, Bc, 1, 2, k);
    if (czp != T(0) || kzp != T(1)) {
      stretch(dzEy, bzp, czp, kzp, ps, v.psi[0]);
      stretch(dzEx, bzp, czp, kzp, ps + 3 * cs, v.psi[3]);
    }
    if (pc.cy != T(0) || pc.ky != T(1)) {
      stretch(dyEz, pc.by, pc.cy, pc.ky, ps + cs, v.psi[1]);
      stretch(dyEx, pc.by, pc.cy, pc.ky, ps + 4 * cs, v.psi[4]);
    }
    if (pc.cx != T(0) || pc.kx != T(1)) {
      stretch(dxEz, pc.bx, pc.cx, pc.kx, ps + 2 * cs, v.psi[2]);
      stretch(dxEy, pc.bx, pc.cx, pc.kx, ps + 5 * cs, v.psi[5]);
    }
  }
  const T db_u = c.db_u, mu_r0 = c.mu_r0;
  T dbx = db_u, dby = db_u, dbz = db_u, mx = mu_r0, my = mu_r0, mz = mu_r0;
  if (GEN && M) {  // node permeability: mean of the (two) cells containing the node
    const int ci0 = clampi(i - 1, 0, nx - 1), ci1 = clampi(i, 0, nx - 1);
    const int cj0 = clampi(j - 1, 0, ny - 1), cj1 = clampi(j, 0, ny - 1);
    const long long cp = (long long)nx * ny;
    const long long c0 = c.coff + ci0 + (long long)nx * cj0 + cp * clampi(k - 1, 0, nz - 1);
    const T A0 = M[c0];
    mx = T(0.5) * (A0 + M[c0 + (ci1 - ci0)]);
    my = T(0.5) * (A0 + M[c0 + (long long)(cj1 - cj0) * nx]);
    mz = T(0.5) * (A0 + M[c.coff + ci0 + (long long)nx * cj0 + cp * clampi(k, 0, nz - 1)]);
    const T dtm0x2 = c.dtm0x2;
    dbx = quot(dtm0x2, mx + mx);
    dby = quot(dtm0x2, my + my);
    dbz = quot(dtm0x2, mz + mz);
  }
  T chx = dzEy - dyEz, chy = dxEz - dzEx, chz = dyEx - dxEy;
  if constexpr (TF) {  // TF/SF corrections (zero off the box surface)
    chx += tcx;
    chy += tcy;
    chz += tcz;
  }
  const T nhx = hx + dbx * chx;
  const T nhy = hy + dby * chy;
  const T nhz = hz + dbz * chz;
  const bool vx = i <= nx, vy = j <= ny, vz = k <= nz;
  if (store && vx) st32(Hx, (unsigned)o, nhx);
  if (store && vy) st32(Hy, (unsigned)o, nhy);
  if (store && vz) st32(Hz, (unsigned)o, nhz);
  onx = nhx;
  ony = nhy;
  onz = nhz;
  if (xin && yin && zin) return mx * (nhx * hx) + my * (nhy * hy) + mz * (nhz * hz);
  const T kxy = (T)wm1(nz, k), kz = vz ? (T)wp1(nz, k) : T(0);
  return (lw.x * kxy) * mx * (nhx * hx) + (lw.y * kxy) * my * (nhy * hy) + (lw.z * kz) * mz * (nhz * hz);
}

// H half step over the tiles [t0, t1) of the tile list (one kind of block),
// each thread marching a node column through the tile's planes, plus the H
// part of W^n:
// 1/2 mu w H^{n+1/2} H^{n-1/2}.  GEN: per-cell permeability or interfaces.
template <typename T, bool GEN, bool IFACE, bool PML, bool TF = false>
__global__ __launch_bounds__(256) void k_h_update(KArgs a) {
  double eacc = 0.0;
  const long long nstep = a.st->step;
  const void* pin = pool_in(a, nstep);
  void* pout = pool_out(a, nstep);
  TileIter it(a.t1 - a.t0, a.order);
  for (int tv; it.next(tv);) {
    const int t = __builtin_amdgcn_readfirstlane(tv) + a.t0;
    const SBP_CONST Tile& tl = as_const(a.tiles)[t];
    const int tb = tl.block, tq0 = tl.q0, tz0 = tl.z0, tflags = tl.pad;
    const DevBlock& B = a.blocks[tb];
    const SBP_CONST DevBlock& Bc = as_const(a.blocks)[tb];
    const BC<T> c(Bc);
    const double kh = Bc.kh;
    const T* base = (const T*)pin + Bc.foff;  // E^n, H^{n-1/2}
    T* bout = (T*)pout + Bc.foff;             // H^{n+1/2}
    const long long csz = Bc.csz;
    const T* M = (GEN && (c.mat & MAT_MU)) ? (const T*)a.mat_mu : nullptr;
    const int q = tq0 + (int)threadIdx.x;
    if (q >= (int)c.sx * (c.ny + 2)) continue;
    const int j = q / (int)c.sx, i = q - j * (int)c.sx;
    const TRow<T> rx = row_of<T>(B, 0, i, true), ry = row_of<T>(B, 1, j, true);  // D- rows of the column
    const W3<T> lw = h_col_weights<T>(c.nx, c.ny, i, j);
    const FaceCol fc = IFACE ? face_col(Bc, i, j, 3) : FaceCol{0, 0};  // D- rows: low face below 3
    const PmlCol<T> pc = PML ? pml_col<T>(a, Bc, 1, i, j) : PmlCol<T>{};
    const int k0 = tz0, k1 = min(tz0 + a.cz, c.nz + 2);
    const T* Ex = base;
    const T* Ey = base + csz;
    const T* Ez = base + 2 * csz;
    const T* Hx = base + 3 * csz;
    const T* Hy = base + 4 * csz;
    const T* Hz = base + 5 * csz;
    T* HxO = bout + 3 * csz;
    T* HyO = bout + 4 * csz;
    T* HzO = bout + 5 * csz;
    double es = 0.0;
    long long o = (long long)q + c.sxy * k0;
    HIn<T> cur;
    {
      const long long ob = k0 > 0 ? o - c.sxy : o;
      cur.ex_z = Ex[ob];
      cur.ey_z = Ey[ob];
      h_load<T>(cur, c, Ex, Ey, Ez, Hx, Hy, Hz, i, j, o);
      if (IFACE && rx.nbr) h_face<T>(a, c, fc, k0, cur);
      if (IFACE && !ry.in) h_yrow<T>(a, c, fc, ry, Ez, Ex, j, k0, o, cur);
      if constexpr (IFACE && sizeof(T) == 4) h_zrow<T>(a, c, Bc, Ey, Ex, i, j, k0, o, cur);
      if constexpr (PML) psi_load<T, false>(a, Bc, pc, k0, o, cur.psi);
    }
    for (int k = k0; k < k1; ++k, o += c.sxy) {
      HIn<T> nxt;
      if (k + 1 < k1) {  // next plane first: its loads overlap this plane's arithmetic
        nxt.ex_z = cur.ex;
        nxt.ey_z = cur.ey;
        h_load<T>(nxt, c, Ex, Ey, Ez, Hx, Hy, Hz, i, j, o + c.sxy);
        if (IFACE && rx.nbr) h_face<T>(a, c, fc, k + 1, nxt);
        if (IFACE && !ry.in) h_yrow<T>(a, c, fc, ry, Ez, Ex, j, k + 1, o + c.sxy, nxt);
        if constexpr (IFACE && sizeof(T) == 4) h_zrow<T>(a, c, Bc, Ey, Ex, i, j, k + 1, o + c.sxy, nxt);
        if constexpr (PML) psi_load<T, false>(a, Bc, pc, k + 1, o + c.sxy, nxt.psi);
      }
      T v0, v1, v2, tcx = T(0), tcy = T(0), tcz = T(0);
      // in place: gathering one plane ahead costs the H kernel a wave per SIMD
      if (TF && (tflags & 4) && tf_near(*as_const(a.tf), i, j, k)) tf_terms<false, T>(a, Bc, i, j, k, tcx, tcy, tcz);
      es += (double)h_node<T, GEN, IFACE, PML, TF>(a, Bc, rx, ry, lw, c, cur, Ex, Ey, Ez, HxO, HyO, HzO, M, fc, pc, tcx,
                                               tcy, tcz, i, j, k, o, true, v0, v1, v2);
      if (tflags & 2) take_probes<T>(a, B, i, j, k, true, nstep, v0, v1, v2);
      cur = nxt;
    }
    eacc += kh * es;
  }
  store_partial(eacc, a);
}

// ------------------------------------------------------------- E update
// The four cells around an E node column at planes k-1 (P0) and k (P1):
// A (i-1, j-1), B (i, j-1), C (i-1, j), D (i, j), clamped to the block; cell
// X of plane P is at index A + P + (offset of X from A).
struct Cells {
  long long A, P0, P1;
  int dx, dy;
};

template <typename T>
__device__ __forceinline__ Cells cells_of(const BC<T>& c, int i, int j, int k) {
  const int nx = c.nx, ny = c.ny, nz = c.nz;
  const long long cp = (long long)nx * ny;
  Cells r;
  if (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1 && k >= 1 && k <= nz - 1) {
    r.A = c.coff + (i - 1) + (long long)nx * (j - 1);
    r.dx = 1;
    r.dy = nx;
    r.P0 = cp * (k - 1);
    r.P1 = r.P0 + cp;
  } else {
    const int ci0 = clampi(i - 1, 0, nx - 1), ci1 = clampi(i, 0, nx - 1);
    const int cj0 = clampi(j - 1, 0, ny - 1), cj1 = clampi(j, 0, ny - 1);
    r.A = c.coff + ci0 + (long long)nx * cj0;
    r.dx = ci1 - ci0;
    r.dy = (cj1 - cj0) * nx;
    r.P0 = cp * clampi(k - 1, 0, nz - 1);
    r.P1 = cp * clampi(k, 0, nz - 1);
  }
  return r;
}

// Sums of a per-cell quantity over the cells containing an Ex, Ey, Ez node
// (four each; the node value is a quarter of the sum).
template <typename T>
struct Sum4 {
  T x, y, z;
};
template <typename T>
__device__ __forceinline__ Sum4<T> cell_sums(const T* __restrict__ M, const Cells& q) {
  const T* p0 = M + q.A + q.P0;
  const T* p1 = M + q.A + q.P1;
  const T a0 = p0[0], b0 = p0[q.dx], c0 = p0[q.dy], d0 = p0[q.dx + q.dy];
  const T a1 = p1[0], b1 = p1[q.dx], c1 = p1[q.dy];
  return Sum4<T>{(a0 + c0) + (a1 + c1), (a0 + b0) + (a1 + b1), (a0 + b0) + (c0 + d0)};
}

// Values one E node update reads at interior rows: E and H at the node, H
// one node ahead along y and x (offsets kept inside the component box on the
// last row / column), Hx, Hy one plane ahead and the permittivity cells of
// planes k-1 (e0*) and k (e1*).  Walking a column of planes, the centre Hx,
// Hy and the plane k-1 cells are the previous plane's values, carried in
// registers; e1d is loaded for the next plane's e0d.
template <typename T>
struct EIn {
  T ex, ey, ez, hx, hy, hz;
  T hy_z, hx_z, hz_y, hx_y, hz_x, hy_x;
  T hz_xx, hy_xx;  // x closure rows: the value beyond the interior pair (e_xd)
  double hz_f, hy_f;  // interface x rows: the neighbour's face values (fp64)
  T hz_yy, hx_yy;     // y rows of interface blocks: likewise
  double hz_fy, hx_fy;
  T e0a, e0b, e0c, e0d, e1a, e1b, e1c, e1d;
  unsigned i1a, i1b, i1c, i1d;  // tabled permittivity: the plane's table indices, looked up when used
  T psi[6];  // absorbing layers: the node's recursion variables (slots 6-11)
};

// Cell offsets of a node column (i, j) within the block's cells: cell A
// (i-1, j-1) clamped, and the offsets of B (+x) and C (+y); plane P of cells
// starts at P * nx * ny.
struct ColCells {
  long long A, cp;
  int dx, dy;
};
template <typename T>
__device__ __forceinline__ ColCells col_cells(const BC<T>& c, int i, int j) {
  const int nx = c.nx, ny = c.ny;
  const int ci0 = clampi(i - 1, 0, nx - 1), ci1 = clampi(i, 0, nx - 1);
  const int cj0 = clampi(j - 1, 0, ny - 1), cj1 = clampi(j, 0, ny - 1);
  return ColCells{ci0 + (long long)nx * cj0, (long long)nx * ny, ci1 - ci0, (cj1 - cj0) * nx};
}

// Permittivity of a plane's four cells from the table indices loaded with it.
template <typename T>
__device__ __forceinline__ void e_cells(EIn<T>& v, const T* etab) {
  v.e1a = etab[v.i1a];
  v.e1b = etab[v.i1b];
  v.e1c = etab[v.i1c];
  v.e1d = etab[v.i1d];
}

// EIDX: the block's cells as byte indices (MI) into its table; the indices
// stay in registers until the plane's other loads are needed too (a lookup
// here would wait for the whole prefetch of the plane).
template <typename T, bool HAS_EPS, bool EIDX = false>
__device__ __forceinline__ void e_load(EIn<T>& v, const BC<T>& c, const T* __restrict__ Ex,
                                       const T* __restrict__ Ey, const T* __restrict__ Ez,
                                       const T* __restrict__ Hz, const T* __restrict__ Hx,
                                       const T* __restrict__ Hy, const T* __restrict__ ME, const ColCells& q,
                                       int i, int j, int k, long long o,
                                       const unsigned char* __restrict__ MI = nullptr) {
  const unsigned u = (unsigned)o;
  const unsigned uz = u + (k <= c.nz ? (unsigned)c.sxy : 0u), uy = u + (j <= c.ny ? (unsigned)c.sx : 0u),
                 ux = u + (i <= c.nx ? 1u : 0u);
  v.ex = ld32(Ex, u);
  v.ey = ld32(Ey, u);
  v.ez = ld32(Ez, u);
  v.hz = ld32(Hz, u);
  v.hy_z = ld32(Hy, uz);
  v.hx_z = ld32(Hx, uz);
  v.hz_y = ld32(Hz, uy);
  v.hx_y = ld32(Hx, uy);
  v.hz_x = ld32(Hz, ux);
  v.hy_x = ld32(Hy, ux);
  const int xd = e_xd(i, c.nx);
  if (xd != 0) {
    v.hz_xx = ld32(Hz, u + (unsigned)xd);
    v.hy_xx = ld32(Hy, u + (unsigned)xd);
  }
  if (HAS_EPS) {  // ME (MI): the block's cells; q.A relative to them
    const unsigned p1 = (unsigned)(q.A + q.cp * clampi(k, 0, c.nz - 1));
    if constexpr (EIDX) {
      v.i1a = MI[p1];
      v.i1b = MI[p1 + (unsigned)q.dx];
      v.i1c = MI[p1 + (unsigned)q.dy];
      v.i1d = MI[p1 + (unsigned)(q.dx + q.dy)];
    } else {
      v.e1a = ld32(ME, p1);
      v.e1b = ld32(ME, p1 + (unsigned)q.dx);
      v.e1c = ld32(ME, p1 + (unsigned)q.dy);
      v.e1d = ld32(ME, p1 + (unsigned)(q.dx + q.dy));
    }
  }
}

// Interface x rows of plane k: the neighbour's face values, the Hz and Hy
// slots of the x face.
template <typename T>
__device__ __forceinline__ void e_face(const KArgs& a, const BC<T>& c, const FaceCol& fc, int k, EIn<T>& v) {
  const long long by = c.ny + 2, fs = by * (c.nz + 2), fo = fc.x + by * k + 2 * fs;
  v.hz_f = a.face[fo + fs];
  v.hy_f = a.face[fo];
}

// The y rows of an interface block at plane k (Hz and Hx slots of the y face).
template <typename T>
__device__ __forceinline__ void e_yrow(const KArgs& a, const BC<T>& c, const FaceCol& fc, const TRow<T>& ry,
                                       const T* __restrict__ Hz, const T* __restrict__ Hx, int j, int k,
                                       long long o, EIn<T>& v) {
  const int yd = e_xd(j, c.ny);
  if (yd != 0) {
    const unsigned u = (unsigned)o + (unsigned)(yd * (int)c.sx);
    v.hz_yy = ld32(Hz, u);
    v.hx_yy = ld32(Hx, u);
  }
  if (ry.nbr) {
    const long long bx = c.nx + 2, fs = bx * (c.nz + 2), fo = fc.y + bx * k + 2 * fs;
    v.hz_fy = a.face[fo + fs];
    v.hx_fy = a.face[fo];
  }
}

// E^{n+1} = Ca E^n + Cb (E7-E9 + J) at node (i, j, k), all valid E
// components, with the closure / PMC / absorbing / interface rows replacing
// the interior differences on the boundary rows; the absorbing damping
// 2/(eta h) on tangential face nodes joins the semi-implicit loss.  Returns
// the node's 4 eps_r (w/h^3) (E^n)^2 (the E part of W^n).
template <typename T, bool HAS_EPS, bool GEN, bool IFACE, bool PML>
__device__ __forceinline__ T e_node(const KArgs& a, const DevBlock& B, const SBP_CONST DevBlock& Bc,
                                    const TRow<T>& rx, const TRow<T>& ry, const W3<T>& lw, const BC<T>& c,
                                    const EIn<T>& v,
                                    T* __restrict__ Ex, T* __restrict__ Ey, T* __restrict__ Ez,
                                    const T* __restrict__ Hx, const T* __restrict__ Hy,
                                    const T* __restrict__ Hz, const T* __restrict__ MS, const FaceCol& fc,
                                    const PmlCol<T>& pc, int i, int j, int k, long long o, T jx, T jy, T jz,
                                    T& onx, T& ony, T& onz) {
  const int nx = c.nx, ny = c.ny, nz = c.nz;
  const long long sx = c.sx, sxy = c.sxy;
  const T ihx = c.ihx, ihy = c.ihy, ihz = c.ihz;
  const bool xin = i >= 2 && i <= nx - 2, yin = j >= 2 && j <= ny - 2, zin = k >= 2 && k <= nz - 2;
  const T ex = v.ex, ey = v.ey, ez = v.ez;
  const T hx = v.hx, hy = v.hy, hz = v.hz;
  T dzHy = (v.hy_z - hy) * ihz, dzHx = (v.hx_z - hx) * ihz;
  T dyHz = (v.hz_y - hz) * ihy, dyHx = (v.hx_y - hx) * ihy;
  T dxHz = (v.hz_x - hz) * ihx, dxHy = (v.hy_x - hy) * ihx;
  // face-buffer slots of tangential H: 2 and 3 (ascending tangential axis)
  const long long bx = nx + 2, by = ny + 2, bz = nz + 2;
  if (!zin) {
    if (k <= nz) {
      const TRow<T> rz = row_of<T>(Bc, 2, k, false);
      const long long fs = bx * by, fo = Bc.fboff[k < 2 ? 4 : 5] + i + bx * j + 2 * fs;
      dzHy = drow<T, IFACE>(a, Hy, o, sxy, rz, fo + fs, Bc.ih[2]);
      dzHx = drow<T, IFACE>(a, Hx, o, sxy, rz, fo, Bc.ih[2]);
    } else {
      dzHy = dzHx = T(0);  // Ex, Ey do not exist on plane nz+1
    }
  }
  if (!yin) {
    if constexpr (IFACE) {
      const int yd = e_xd(j, ny);
      dyHz = xrow<T>(ry, v.hz, v.hz_y, 1, v.hz_yy, yd);
      dyHx = xrow<T>(ry, v.hx, v.hx_y, 1, v.hx_yy, yd);
      if (ry.nbr) {
        dyHz = pen<T>(dyHz, ry.cn, Bc.ih[1], v.hz_fy);
        dyHx = pen<T>(dyHx, ry.cn, Bc.ih[1], v.hx_fy);
      }
    } else {
      const long long fs = bx * bz, fo = fc.y + bx * k + 2 * fs;
      dyHz = drow<T, IFACE>(a, Hz, o, sx, ry, fo + fs, Bc.ih[1]);
      dyHx = drow<T, IFACE>(a, Hx, o, sx, ry, fo, Bc.ih[1]);
    }
  }
  if (!xin) {
    const int xd = e_xd(i, nx);
    dxHz = xrow<T>(rx, v.hz, v.hz_x, 1, v.hz_xx, xd);
    dxHy = xrow<T>(rx, v.hy, v.hy_x, 1, v.hy_xx, xd);
    if (IFACE && rx.nbr) {
      dxHz = pen<T>(dxHz, rx.cn, Bc.ih[0], v.hz_f);
      dxHy = pen<T>(dxHy, rx.cn, Bc.ih[0], v.hy_f);
    }
  }
  if constexpr (PML) {  // absorbing layers: E terms sit on the "+" grid of their axis
    T* ps = (T*)a.psi + Bc.psi_off + 6 * Bc.csz + o;  // slots 6-11: (Ex,y) (Ex,z) (Ey,z) (Ey,x) (Ez,x) (Ez,y)
    const long long cs = Bc.csz;
    if (k <= nz) {
      const T bzp = pml_z<T>(a, Bc, 0, 0, k), czp = pml_z<T>(a, Bc, 0, 1, k), kzp = pml_z<T>(a, Bc, 0, 2, k);
      if (czp != T(0) || kzp != T(1)) {
        stretch(dzHy, bzp, czp, kzp, ps + cs, v.psi[1]);
        stretch(dzHx, bzp, czp, kzp, ps + 2 * cs, v.psi[2]);
      }
    }
    if (pc.cy != T(0) || pc.ky != T(1)) {
      stretch(dyHz, pc.by, pc.cy, pc.ky, ps, v.psi[0]);
      stretch(dyHx, pc.by, pc.cy, pc.ky, ps + 5 * cs, v.psi[5]);
    }
    if (pc.cx != T(0) || pc.kx != T(1)) {
      stretch(dxHz, pc.bx, pc.cx, pc.kx, ps + 3 * cs, v.psi[3]);
      stretch(dxHy, pc.bx, pc.cx, pc.kx, ps + 4 * cs, v.psi[4]);
    }
  }
  const T cx = dyHz - dzHy, cy = dzHx - dxHz, cz = dxHy - dyHx;
  const T eps_r0 = c.eps_r0;
  T mx = T(4) * eps_r0, my = mx, mz = mx;  // node permittivity x4: sums of the four containing cells
  if (HAS_EPS) {
    mx = (v.e0a + v.e0c) + (v.e1a + v.e1c);
    my = (v.e0a + v.e0b) + (v.e1a + v.e1b);
    mz = (v.e0a + v.e0b) + (v.e0c + v.e0d);
  }
  T cax = T(1), cay = T(1), caz = T(1), cbx, cby, cbz;
  if (HAS_EPS) {
    const T dte0x4 = c.dte0x4;
    cbx = quot(dte0x4, mx);
    cby = quot(dte0x4, my);
    cbz = quot(dte0x4, mz);
  } else {
    cbx = cby = cbz = c.cb_u;
  }
  if (GEN) {
    const int am = c.abc;
    const T gx = (T)((int)(i == 0 && (am & 1)) + (int)(i == nx && (am & 2))) * ihx;
    const T gy = (T)((int)(j == 0 && (am & 4)) + (int)(j == ny && (am & 8))) * ihy;
    const T gz = (T)((int)(k == 0 && (am & 16)) + (int)(k == nz && (am & 32))) * ihz;
    const T gEx = gy + gz, gEy = gx + gz, gEz = gx + gy;
    const bool lossy = MS != nullptr || c.sig0 != T(0);
    if (lossy || gEx != T(0) || gEy != T(0) || gEz != T(0)) {
      // b = dt (sigma + sigma_abc) / (2 eps), sigma_abc = 2 g / eta, eta = sqrt(mu/eps);
      // Ca = (1-b)/(1+b), Cb = (dt/eps)/(1+b)
      const T sig0 = c.sig0;
      T sx4 = T(4) * sig0, sy4 = sx4, sz4 = sx4;
      if (MS) {
        const Sum4<T> q = cell_sums(MS, cells_of(c, i, j, k));
        sx4 = q.x;
        sy4 = q.y;
        sz4 = q.z;
      }
      if (gEx != T(0) || gEy != T(0) || gEz != T(0)) {
        T mux = T(4) * (T)B.mu_r0, muy = mux, muz = mux;  // node mu_r x4
        if (c.mat & MAT_MU) {
          const Sum4<T> q = cell_sums((const T*)a.mat_mu, cells_of(c, i, j, k));
          mux = q.x;
          muy = q.y;
          muz = q.z;
        }
        const T me0 = (T)(a.mu0 / a.eps0);
        if (gEx != T(0)) sx4 += T(8) * gEx / sqrt(me0 * mux / mx);
        if (gEy != T(0)) sy4 += T(8) * gEy / sqrt(me0 * muy / my);
        if (gEz != T(0)) sz4 += T(8) * gEz / sqrt(me0 * muz / mz);
      }
      const T hdte0 = c.hdte0, dte0x4 = c.dte0x4;
      const T bx = quot(hdte0 * sx4, mx), by = quot(hdte0 * sy4, my), bz = quot(hdte0 * sz4, mz);
      const T rxx = quot(T(1), T(1) + bx), ryy = quot(T(1), T(1) + by), rzz = quot(T(1), T(1) + bz);
      cax = (T(1) - bx) * rxx;
      cay = (T(1) - by) * ryy;
      caz = (T(1) - bz) * rzz;
      cbx = quot(dte0x4, mx) * rxx;
      cby = quot(dte0x4, my) * ryy;
      cbz = quot(dte0x4, mz) * rzz;
    }
  }
  const T nex = cax * ex + cbx * (cx + jx);
  const T ney = cay * ey + cby * (cy + jy);
  const T nez = caz * ez + cbz * (cz + jz);
  const bool vz = k <= nz;
  const bool vEx = j <= ny && vz, vEy = i <= nx && vz, vEz = i <= nx && j <= ny;
  if (vEx) st32(Ex, (unsigned)o, nex);
  if (vEy) st32(Ey, (unsigned)o, ney);
  if (vEz) st32(Ez, (unsigned)o, nez);
  onx = nex;
  ony = ney;
  onz = nez;
  // norm weights / h: 1 inside, Appendix P+ / P- on the boundary rows
  const T kxy = vz ? (T)wp1(nz, k) : T(0), kz = (T)wm1(nz, k);
  {
    // rounded product by product, so that the value does not depend on
    // which kernel variant the compiler fuses into multiply-adds
#pragma clang fp contract(off)
    return (lw.x * kxy) * mx * (ex * ex) + (lw.y * kxy) * my * (ey * ey) + (lw.z * kz) * mz * (ez * ez);
  }
}

// E step over the tiles [t0, t1) of the tile list (one kind of block): each
// thread marches a node column through the tile's planes.  The workgroup
// adds the E part of W^n, 1/2 eps w (E^n)^2 (E^n being the centre values it
// loads anyway), to the H partial of the same tile from the H launch; the
// finish kernel then writes W^n to energy slot n and advances the step
// index.  GEN: loss, absorbing faces, per-cell permeability or interfaces.
// Waves per SIMD the E kernels are held to (1: no bound): the tabled fp32
// variant would take 97 VGPRs (4 waves) unbounded and fits 5 waves in 95.
// (The plain fp64 variants take 141-143 VGPRs, 3 waves; held to 4 they
// spill 12-20 B per lane and run 1% slower.)
template <typename T, bool GENERAL, bool EIDX>
constexpr int e_waves() {
  return (!GENERAL && EIDX && sizeof(T) == 4) ? 5 : 1;
}

// EIDX: plain blocks with per-cell permittivity whose cells take at most
// kCellTab values read one byte per cell and look the value up in the
// block's table.  Each wave keeps its own copy of the table in LDS, written
// by its 64 lanes whenever its tile changes block (before any lane leaves
// the tile) and read back by the same wave: LDS operations of one wave
// complete in order, so no workgroup barrier holds the other waves.
template <typename T, bool HAS_EPS, bool GEN, bool IFACE, bool PML, bool TF = false, bool EIDX = false>
__global__ __launch_bounds__(256, (e_waves<T, (GEN || IFACE || PML || TF), EIDX>())) void k_e_update(KArgs a) {
  double eacc = 0.0;
  const long long nstep = a.st->step;
  const void* pin = pool_in(a, nstep);
  void* pout = pool_out(a, nstep);
  static_assert(kCellTab == 64, "one table entry per lane of a wave64");
  __shared__ T wtabs[EIDX ? 4 : 1][EIDX ? kCellTab : 1];  // one table per wave (at most 256 threads)
  T* etab = wtabs[EIDX ? (threadIdx.x >> 6) : 0];
  int tab_block = -1;
  TileIter it(a.t1 - a.t0, a.order);
  for (int tv; it.next(tv);) {
    const int t = __builtin_amdgcn_readfirstlane(tv) + a.t0;
    const SBP_CONST Tile& tl = as_const(a.tiles)[t];
    const int tb = tl.block, tq0 = tl.q0, tz0 = tl.z0, tflags = tl.pad;
    if constexpr (EIDX) {
      if (tb != tab_block) {  // uniform: the workgroup walks one tile sequence
        etab[threadIdx.x & 63] = ((const T*)a.mat_tab)[(long long)tb * kCellTab + (threadIdx.x & 63)];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        tab_block = tb;
      }
    }
    const DevBlock& B = a.blocks[tb];
    const SBP_CONST DevBlock& Bc = as_const(a.blocks)[tb];
    const BC<T> c(Bc);
    const double ke4 = 0.25 * Bc.ke;
    const T* base = (const T*)pin + Bc.foff;  // E^n
    T* bout = (T*)pout + Bc.foff;             // H^{n+1/2} (read), E^{n+1} (written)
    const long long csz = Bc.csz;
    const T* ME = (HAS_EPS && !EIDX) ? (const T*)a.mat_eps + Bc.coff : nullptr;  // the block's permittivity cells
    const unsigned char* MI = EIDX ? a.mat_idx + Bc.coff : nullptr;             // or their table indices
    const T* MS = (GEN && (c.mat & MAT_SIG)) ? (const T*)a.mat_sig : nullptr;
    const int q = tq0 + (int)threadIdx.x;
    if (q >= (int)c.sx * (c.ny + 2)) continue;
    const int j = q / (int)c.sx, i = q - j * (int)c.sx;
    const TRow<T> rx = row_of<T>(B, 0, i, false), ry = row_of<T>(B, 1, j, false);  // D+ rows of the column
    const W3<T> lw = e_col_weights<T>(c.nx, c.ny, i, j);
    const FaceCol fc = IFACE ? face_col(Bc, i, j, 2) : FaceCol{0, 0};  // D+ rows: low face below 2
    const PmlCol<T> pc = PML ? pml_col<T>(a, Bc, 0, i, j) : PmlCol<T>{};
    const int k0 = tz0, k1 = min(tz0 + a.cz, c.nz + 2);
    const T* Ex = base;
    const T* Ey = base + csz;
    const T* Ez = base + 2 * csz;
    const T* Hx = bout + 3 * csz;
    const T* Hy = bout + 4 * csz;
    const T* Hz = bout + 5 * csz;
    T* ExO = bout;
    T* EyO = bout + csz;
    T* EzO = bout + 2 * csz;
    const ColCells cc = col_cells(c, i, j);
    double es = 0.0;
    long long o = (long long)q + c.sxy * k0;
    EIn<T> cur;
    cur.hx = Hx[o];
    cur.hy = Hy[o];
    if (HAS_EPS) {
      const unsigned p0 = (unsigned)(cc.A + cc.cp * clampi(k0 - 1, 0, c.nz - 1));
      if constexpr (EIDX) {
        cur.e0a = etab[MI[p0]];
        cur.e0b = etab[MI[p0 + (unsigned)cc.dx]];
        cur.e0c = etab[MI[p0 + (unsigned)cc.dy]];
        cur.e0d = etab[MI[p0 + (unsigned)(cc.dx + cc.dy)]];
      } else {
        cur.e0a = ME[p0];
        cur.e0b = ME[p0 + (unsigned)cc.dx];
        cur.e0c = ME[p0 + (unsigned)cc.dy];
        cur.e0d = ME[p0 + (unsigned)(cc.dx + cc.dy)];
      }
    }
    e_load<T, HAS_EPS, EIDX>(cur, c, Ex, Ey, Ez, Hz, Hx, Hy, ME, cc, i, j, k0, o, MI);
    if (IFACE && rx.nbr) e_face<T>(a, c, fc, k0, cur);
    if (IFACE && !ry.in) e_yrow<T>(a, c, fc, ry, Hz, Hx, j, k0, o, cur);
    if constexpr (PML) psi_load<T, true>(a, Bc, pc, k0, o, cur.psi);
    TfPre tcur, tnxt;
    if (TF && (tflags & 4)) tf_gather<true>(a, i, j, k0, tcur);
    for (int k = k0; k < k1; ++k, o += c.sxy) {
      EIn<T> nxt;
      if (k + 1 < k1) {  // next plane first: its loads overlap this plane's arithmetic
        e_load<T, HAS_EPS, EIDX>(nxt, c, Ex, Ey, Ez, Hz, Hx, Hy, ME, cc, i, j, k + 1, o + c.sxy, MI);
        if (IFACE && rx.nbr) e_face<T>(a, c, fc, k + 1, nxt);
        if (IFACE && !ry.in) e_yrow<T>(a, c, fc, ry, Hz, Hx, j, k + 1, o + c.sxy, nxt);
        if constexpr (PML) psi_load<T, true>(a, Bc, pc, k + 1, o + c.sxy, nxt.psi);
        if (TF && (tflags & 4)) tf_gather<true>(a, i, j, k + 1, tnxt);
      }
      if constexpr (EIDX) e_cells(cur, etab);  // this plane's cells, their indices loaded with the plane
      nxt.hx = cur.hx_z;  // carried to the next plane
      nxt.hy = cur.hy_z;
      nxt.e0a = cur.e1a;
      nxt.e0b = cur.e1b;
      nxt.e0c = cur.e1c;
      nxt.e0d = cur.e1d;
      T jx = T(0), jy = T(0), jz = T(0);
      if (tflags & 1) source_terms<T>(a, B, i, j, k, jx, jy, jz);
      if (TF && (tflags & 4)) tf_combine<true, T>(a, Bc, tcur, jx, jy, jz);
      T v0, v1, v2;
      es += (double)e_node<T, HAS_EPS, GEN, IFACE, PML>(a, B, Bc, rx, ry, lw, c, cur, ExO, EyO, EzO, Hx, Hy, Hz, MS, fc,
                                                        pc, i, j, k, o, jx, jy, jz, v0, v1, v2);
      if (tflags & 2) take_probes<T>(a, B, i, j, k, false, nstep, v0, v1, v2);
      cur = nxt;
      if (TF) tcur = tnxt;
    }
    eacc += ke4 * es;
  }
  store_partial(eacc, a);
}

// ------------------------------------------------------------ one-pass step
// For plain blocks (PEC / PMC faces, per-cell or uniform permittivity) both
// half steps run in one pass: a workgroup takes a 32 x 8 window of node
// columns and walks up through the planes.  At plane kh it forms H^{n+1/2}
// on the whole window (the same rows as k_h_update) and keeps it in LDS; E
// at plane kh-2 then takes its in-plane neighbours of H^{n+1/2} from LDS and
// its z neighbours (planes kh-3 .. kh) from registers, so the D+ closure rows
// (which reach one node back and two ahead) are local too.  Each field value
// is read once and written once per step; the window's unowned columns (one
// halo column and row) only supply H neighbours.
template <typename T>
__device__ __forceinline__ T lds_h(const T (&hs)[4][3][FY][FX], int slot, int comp, int w, int lane) {
  return hs[slot][comp][min(max(w, 0), FY - 1)][min(max(lane, 0), FX - 1)];
}

// D+ closure row along x (axis 0) or y (axis 1) from the LDS plane.
template <typename T>
__device__ __forceinline__ T lds_row(const T (&hs)[4][3][FY][FX], int slot, int comp, int w, int lane, int axis,
                                     const TRow<T>& R) {
  const int dl = axis == 0 ? 1 : 0, dw = axis == 1 ? 1 : 0;
  const int l0 = lane + dl * R.s, w0 = w + dw * R.s;
  return R.c0 * lds_h(hs, slot, comp, w0, l0) + R.c1 * lds_h(hs, slot, comp, w0 + dw, l0 + dl) +
         R.c2 * lds_h(hs, slot, comp, w0 + 2 * dw, l0 + 2 * dl);
}

// One of the own-column values H(k-1), H(k), H(k+1), H(k+2) by offset d.
template <typename T>
__device__ __forceinline__ T pick4(int d, T m1, T z0, T p1, T p2) {
  return d <= -1 ? m1 : (d == 0 ? z0 : (d == 1 ? p1 : p2));
}

template <typename T, bool HAS_EPS>
__global__ __launch_bounds__(FX * FY) void k_fused(KArgs a) {
  __shared__ T hs[4][3][FY][FX];  // H^{n+1/2} of the last four planes: [plane & 3][comp][row][column]
  double eacc = 0.0;
  const long long nstep = a.st->step;
  const void* pin = pool_in(a, nstep);
  void* pout = pool_out(a, nstep);
  const int lane = threadIdx.x & (FX - 1), w = threadIdx.x / FX;
  TileIter it(a.t1 - a.t0, a.order);
  for (int tv; it.next(tv);) {
    const int t = __builtin_amdgcn_readfirstlane(tv) + a.t0;
    const SBP_CONST FTile& ft = as_const(a.ftiles)[t];
    const int tb = ft.block, z0 = ft.z0, z1 = ft.z1, tflags = ft.flags;
    const DevBlock& B = a.blocks[tb];
    const SBP_CONST DevBlock& Bc = as_const(a.blocks)[tb];
    const BC<T> c(Bc);
    const double kh_e = Bc.kh, ke4 = 0.25 * Bc.ke;
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const int sx = (int)c.sx;
    const long long sxy = c.sxy, csz = Bc.csz;
    const T* base = (const T*)pin + Bc.foff;
    T* bout = (T*)pout + Bc.foff;
    const T* Ex = base;
    const T* Ey = base + csz;
    const T* Ez = base + 2 * csz;
    const T* Hx = base + 3 * csz;
    const T* Hy = base + 4 * csz;
    const T* Hz = base + 5 * csz;
    T* ExO = bout;
    T* EyO = bout + csz;
    T* EzO = bout + 2 * csz;
    T* HxO = bout + 3 * csz;
    T* HyO = bout + 4 * csz;
    T* HzO = bout + 5 * csz;
    const T* ME = HAS_EPS ? (const T*)a.mat_eps + Bc.coff : nullptr;  // the block's permittivity cells
    const int i = ft.i0 + lane, j = ft.j0 + w;
    const bool col = i < sx && j < ny + 2;
    const bool own = col && i >= ft.olx && i <= ft.ohx && j >= ft.oly && j <= ft.ohy;
    const long long oc = col ? (long long)i + (long long)sx * j : 0;
    const ColCells cc = col_cells(c, col ? i : 0, col ? j : 0);
    const TRow<T> hrx = row_of<T>(B, 0, col ? i : 0, true), hry = row_of<T>(B, 1, col ? j : 0, true);
    const W3<T> hlw = h_col_weights<T>(nx, ny, col ? i : 0, col ? j : 0);
    const T ihx = c.ihx, ihy = c.ihy, ihz = c.ihz;
    // own column: Hx, Hy of H^{n+1/2} at planes kh-3 .. kh, E^n at kh-2, kh-1
    T hx3 = T(0), hx2 = T(0), hx1 = T(0), hx0 = T(0), hy3 = T(0), hy2 = T(0), hy1 = T(0), hy0 = T(0);
    T e2x = T(0), e2y = T(0), e2z = T(0), e1x = T(0), e1y = T(0), e1z = T(0);
    T q0a = T(0), q0b = T(0), q0c = T(0), q0d = T(0);  // permittivity cells of plane ke-1
    T q1a = T(0), q1b = T(0), q1c = T(0), q1d = T(0);  // and of plane ke
    if (HAS_EPS && col) {
      const T* p0 = ME + cc.A + cc.cp * clampi(z0 - 1, 0, nz - 1);
      q0a = p0[0];
      q0b = p0[cc.dx];
      q0c = p0[cc.dy];
      q0d = p0[cc.dx + cc.dy];
      const T* p1 = ME + cc.A + cc.cp * clampi(z0, 0, nz - 1);
      q1a = p1[0];
      q1b = p1[cc.dx];
      q1c = p1[cc.dy];
      q1d = p1[cc.dx + cc.dy];
    }
    const int kh_last = min(z1 + 2, nz + 1);  // last H plane of the tile
    // inputs of the H plane, loaded one plane ahead of its use
    HIn<T> vn;
    if (col) {
      const long long o = oc + sxy * z0;
      h_load<T>(vn, c, Ex, Ey, Ez, Hx, Hy, Hz, i, j, o);
      vn.ex_z = z0 > 0 ? Ex[o - sxy] : vn.ex;
      vn.ey_z = z0 > 0 ? Ey[o - sxy] : vn.ey;
    }
    for (int kh = z0; kh <= z1 + 2; ++kh) {
      const int slot = kh & 3;
      const HIn<T> v = vn;
      if (col && kh + 1 <= kh_last) {  // next plane's loads overlap this plane's work
        const long long o = oc + sxy * (kh + 1);
        h_load<T>(vn, c, Ex, Ey, Ez, Hx, Hy, Hz, i, j, o);
        vn.ex_z = v.ex;
        vn.ey_z = v.ey;
      }
      T nhx = T(0), nhy = T(0), nhz = T(0), ex = T(0), ey = T(0), ez = T(0);
      if (col && kh <= kh_last) {
        const long long o = oc + sxy * kh;
        const bool hown = own && kh <= z1;
        T v0, v1, v2;
        const T eh = h_node<T, false, false, false>(a, Bc, hrx, hry, hlw, c, v, Ex, Ey, Ez, HxO, HyO, HzO, nullptr,
                                                    FaceCol{0, 0}, PmlCol<T>{}, T(0), T(0), T(0), i, j, kh, o, hown,
                                                    v0, v1, v2);
        if (hown) {
          eacc += kh_e * (double)eh;
          if (tflags & 2) take_probes<T>(a, B, i, j, kh, true, nstep, v0, v1, v2);
        }
        nhx = v0;
        nhy = v1;
        nhz = v2;
        ex = v.ex;
        ey = v.ey;
        ez = v.ez;
      }
      hx3 = hx2;
      hx2 = hx1;
      hx1 = hx0;
      hx0 = nhx;
      hy3 = hy2;
      hy2 = hy1;
      hy1 = hy0;
      hy0 = nhy;
      hs[slot][0][w][lane] = nhx;
      hs[slot][1][w][lane] = nhy;
      hs[slot][2][w][lane] = nhz;
      // permittivity cells of the next E plane (ke + 1 = kh - 1), loaded ahead
      T r1a = q1a, r1b = q1b, r1c = q1c, r1d = q1d;
      if (HAS_EPS && col && kh - 1 > z0) {
        const T* p1 = ME + cc.A + cc.cp * clampi(kh - 1, 0, nz - 1);
        r1a = p1[0];
        r1b = p1[cc.dx];
        r1c = p1[cc.dy];
        r1d = p1[cc.dx + cc.dy];
      }
      __syncthreads();
      const int ke = kh - 2;
      if (ke >= z0) {
        if (own) {
          const int sl = ke & 3;  // LDS slot of plane ke
          const T hx = hx2, hy = hy2, hz = hs[sl][2][w][lane];
          T dyHz = (lds_h(hs, sl, 2, w + 1, lane) - hz) * ihy;
          T dyHx = (lds_h(hs, sl, 0, w + 1, lane) - hx) * ihy;
          T dxHz = (lds_h(hs, sl, 2, w, lane + 1) - hz) * ihx;
          T dxHy = (lds_h(hs, sl, 1, w, lane + 1) - hy) * ihx;
          T dzHy = (hy1 - hy) * ihz, dzHx = (hx1 - hx) * ihz;
          const bool xin = i >= 2 && i <= nx - 2, yin = j >= 2 && j <= ny - 2, zin = ke >= 2 && ke <= nz - 2;
          if (!zin) {
            if (ke <= nz) {
              const TRow<T> rz = row_of<T>(B, 2, ke, false);
              dzHy = rz.c0 * pick4(rz.s, hy3, hy2, hy1, hy0) + rz.c1 * pick4(rz.s + 1, hy3, hy2, hy1, hy0) +
                     rz.c2 * pick4(rz.s + 2, hy3, hy2, hy1, hy0);
              dzHx = rz.c0 * pick4(rz.s, hx3, hx2, hx1, hx0) + rz.c1 * pick4(rz.s + 1, hx3, hx2, hx1, hx0) +
                     rz.c2 * pick4(rz.s + 2, hx3, hx2, hx1, hx0);
            } else {
              dzHy = dzHx = T(0);  // Ex, Ey do not exist on plane nz+1
            }
          }
          if (!yin) {
            const TRow<T> ry = row_of<T>(B, 1, j, false);
            dyHz = lds_row(hs, sl, 2, w, lane, 1, ry);
            dyHx = lds_row(hs, sl, 0, w, lane, 1, ry);
          }
          if (!xin) {
            const TRow<T> rx = row_of<T>(B, 0, i, false);
            dxHz = lds_row(hs, sl, 2, w, lane, 0, rx);
            dxHy = lds_row(hs, sl, 1, w, lane, 0, rx);
          }
          const T cx = dyHz - dzHy, cy = dzHx - dxHz, cz = dxHy - dyHx;
          T mx = T(4) * c.eps_r0, my = mx, mz = mx;
          T cbx, cby, cbz;
          if (HAS_EPS) {
            mx = (q0a + q0c) + (q1a + q1c);
            my = (q0a + q0b) + (q1a + q1b);
            mz = (q0a + q0b) + (q0c + q0d);
            cbx = quot(c.dte0x4, mx);
            cby = quot(c.dte0x4, my);
            cbz = quot(c.dte0x4, mz);
          } else {
            cbx = cby = cbz = c.cb_u;
          }
          T jx = T(0), jy = T(0), jz = T(0);
          if (tflags & 1) source_terms<T>(a, B, i, j, ke, jx, jy, jz);
          const T nex = e2x + cbx * (cx + jx);
          const T ney = e2y + cby * (cy + jy);
          const T nez = e2z + cbz * (cz + jz);
          const bool vz = ke <= nz;
          const bool vEx = j <= ny && vz, vEy = i <= nx && vz, vEz = i <= nx && j <= ny;
          const long long o = oc + sxy * ke;
          if (vEx) ExO[o] = nex;
          if (vEy) EyO[o] = ney;
          if (vEz) EzO[o] = nez;
          const T wx = vEx ? (T)(wm1(nx, i) * wp1(ny, j) * wp1(nz, ke)) : T(0);
          const T wy = vEy ? (T)(wp1(nx, i) * wm1(ny, j) * wp1(nz, ke)) : T(0);
          const T wz = vEz ? (T)(wp1(nx, i) * wp1(ny, j) * wm1(nz, ke)) : T(0);
          eacc += ke4 * (double)(wx * mx * (e2x * e2x) + wy * my * (e2y * e2y) + wz * mz * (e2z * e2z));
          if (tflags & 2) take_probes<T>(a, B, i, j, ke, false, nstep, nex, ney, nez);
        }
        q0a = q1a;
        q0b = q1b;
        q0c = q1c;
        q0d = q1d;
        q1a = r1a;
        q1b = r1b;
        q1c = r1c;
        q1d = r1d;
      }
      e2x = e1x;
      e2y = e1y;
      e2z = e1z;
      e1x = ex;
      e1y = ey;
      e1z = ez;
    }
    __syncthreads();  // the next tile rewrites the LDS planes
  }
  store_partial(eacc, a);
}

// ------------------------------------------------------- interface gather
// Fills the face buffers: for every own face node, the neighbour's
// tangential field on its coincident face, through the per-axis taps
// (identity at 1:1; the norm-compatible 1:2 interpolation otherwise).
// Accumulated in fp64.
template <typename T>
__global__ __launch_bounds__(256) void k_face_gather(const DevBlock* blocks, const FaceJob* jobs,
                                                     const GatherWG* wgs, const Taps* taps, const void* pool0,
                                                     const void* pool1, const StepState* stp, int from_out,
                                                     double* face) {
  // E^n lives in the pool step n reads, H^{n+1/2} in the one it writes
  const long long n = stp->step;
  const void* pool = ((n & 1) != from_out) ? pool1 : pool0;
  const GatherWG W = wgs[blockIdx.x];
  const FaceJob J = jobs[W.job];
  const DevBlock& B = blocks[J.block];
  const DevBlock& N = blocks[J.nb];
  const long long id = (long long)W.first + threadIdx.x;
  const long long tot = (long long)J.ext[0] * J.ext[1];
  if (id >= tot) return;
  const int r0 = (int)(id % J.ext[0]), r1 = (int)(id / J.ext[0]);
  const long long st[3] = {1, N.sx, N.sxy};
  const int axis = J.face >> 1;
  const long long onrm = (long long)J.nb_idx * st[axis];
  const long long s0 = st[J.t_axis[0]], s1 = st[J.t_axis[1]];
  double v;
  if (J.unit) {  // same mesh: the coincident node itself
    const long long o = onrm + (long long)r0 * s0 + (long long)r1 * s1;
    v = J.w1 * (double)((const T*)pool + N.foff + (long long)J.comp * N.csz)[o];
    if (J.nb2 >= 0) {
      const DevBlock& M = blocks[J.nb2];
      v += J.w2 * (double)((const T*)pool + M.foff + (long long)J.comp * M.csz)[o];
    }
  } else {
    const Taps& T0 = taps[J.taps_off[0] + r0];
    const Taps& T1 = taps[J.taps_off[1] + r1];
    // the interpolated face value of one source block (nb2 has nb's geometry)
    auto gather = [&](const DevBlock& S) {
      const T* nf = (const T*)pool + S.foff + (long long)J.comp * S.csz;
      double acc = 0.0;
      for (int q = 0; q < T1.count; ++q) {
        double sum = 0.0;
        const long long o1 = onrm + (long long)(T1.start + q) * s1;
        for (int p = 0; p < T0.count; ++p) sum += T0.w[p] * (double)nf[o1 + (long long)(T0.start + p) * s0];
        acc += T1.w[q] * sum;
      }
      return acc;
    };
    v = J.w1 * gather(N);
    if (J.nb2 >= 0) v += J.w2 * gather(blocks[J.nb2]);
  }
  // own face-node index in the node-box face layout
  const int bx = B.n[0] + 2, by = B.n[1] + 2;
  long long fidx;
  if (axis == 0) fidx = (long long)r0 + (long long)by * r1;       // (j, k)
  else fidx = (long long)r0 + (long long)bx * r1;                 // (i, k) or (i, j)
  face[B.fboff[J.face] + (long long)(J.is_h * 2 + J.slot) * B.fsz[J.face] + fidx] = v;
}

// ------------------------------------------------------------- launchers
// kind bit 0: per-cell permittivity; bit 1: general block (loss, absorbing
// faces, per-cell permeability, absorbing layers or the TF/SF box); bit 2:
// interface faces (periodic faces included); bit 3: absorbing layers; bit 4:
// the TF/SF box; bit 5: permittivity cells held as byte indices into the
// block's table (plain blocks only: kind 33).  Bits 3 and 4 imply bit 1; bit
// 2 alone (lossless interface blocks) takes the interface rows without the
// general terms.
template <typename T>
hipError_t launch_h(const KArgs& a, int kind, int grid, int threads, hipStream_t s) {
  const dim3 g(grid), b(threads);
  switch (kind & 30) {
    case 0: hipLaunchKernelGGL((k_h_update<T, false, false, false>), g, b, 0, s, a); break;
    case 18: hipLaunchKernelGGL((k_h_update<T, true, false, false, true>), g, b, 0, s, a); break;
    case 26: hipLaunchKernelGGL((k_h_update<T, true, false, true, true>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_h_update<T, true, false, false>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_h_update<T, false, true, false>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_h_update<T, true, true, false>), g, b, 0, s, a); break;
    case 10: hipLaunchKernelGGL((k_h_update<T, true, false, true>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_h_update<T, true, true, true>), g, b, 0, s, a); break;
  }
  return hipGetLastError();
}
template <typename T>
hipError_t launch_e(const KArgs& a, int kind, int grid, int threads, hipStream_t s) {
  const dim3 g(grid), b(threads);
  if (kind == 33) {  // plain, per-cell permittivity from a table
    hipLaunchKernelGGL((k_e_update<T, true, false, false, false, false, true>), g, b, 0, s, a);
    return hipGetLastError();
  }
  switch (kind & 31) {
    case 0: hipLaunchKernelGGL((k_e_update<T, false, false, false, false>), g, b, 0, s, a); break;
    case 18: hipLaunchKernelGGL((k_e_update<T, false, true, false, false, true>), g, b, 0, s, a); break;
    case 19: hipLaunchKernelGGL((k_e_update<T, true, true, false, false, true>), g, b, 0, s, a); break;
    case 26: hipLaunchKernelGGL((k_e_update<T, false, true, false, true, true>), g, b, 0, s, a); break;
    case 27: hipLaunchKernelGGL((k_e_update<T, true, true, false, true, true>), g, b, 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_e_update<T, true, false, false, false>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_e_update<T, false, true, false, false>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_e_update<T, true, true, false, false>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_e_update<T, false, false, true, false>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((k_e_update<T, true, false, true, false>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_e_update<T, false, true, true, false>), g, b, 0, s, a); break;
    case 7: hipLaunchKernelGGL((k_e_update<T, true, true, true, false>), g, b, 0, s, a); break;
    case 10: hipLaunchKernelGGL((k_e_update<T, false, true, false, true>), g, b, 0, s, a); break;
    case 11: hipLaunchKernelGGL((k_e_update<T, true, true, false, true>), g, b, 0, s, a); break;
    case 14: hipLaunchKernelGGL((k_e_update<T, false, true, true, true>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((k_e_update<T, true, true, true, true>), g, b, 0, s, a); break;
  }
  return hipGetLastError();
}
template <typename T>
hipError_t launch_fused(const KArgs& a, int kind, int grid, hipStream_t s) {
  if (kind & 1) hipLaunchKernelGGL((k_fused<T, true>), dim3(grid), dim3(FX * FY), 0, s, a);
  else hipLaunchKernelGGL((k_fused<T, false>), dim3(grid), dim3(FX * FY), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_fused<float>(const KArgs&, int, int, hipStream_t);
template hipError_t launch_fused<double>(const KArgs&, int, int, hipStream_t);

hipError_t launch_finish(const KArgs& a, int p0, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, a, p0, nparts);
  return hipGetLastError();
}
hipError_t launch_sources(const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_sources, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_gather(const DevBlock* blocks, const FaceJob* jobs, const GatherWG* wgs, int nwg,
                         const Taps* taps, const KArgs& a, int from_out, double* face, hipStream_t s) {
  if (nwg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_face_gather<T>, dim3(nwg), dim3(256), 0, s, blocks, jobs, wgs, taps, a.pool, a.pool2, a.st,
                     from_out, face);
  return hipGetLastError();
}

template hipError_t launch_h<float>(const KArgs&, int, int, int, hipStream_t);
template hipError_t launch_h<double>(const KArgs&, int, int, int, hipStream_t);
template hipError_t launch_e<float>(const KArgs&, int, int, int, hipStream_t);
template hipError_t launch_e<double>(const KArgs&, int, int, int, hipStream_t);
template hipError_t launch_gather<float>(const DevBlock*, const FaceJob*, const GatherWG*, int, const Taps*, const KArgs&, int,
                                        double*, hipStream_t);
template hipError_t launch_gather<double>(const DevBlock*, const FaceJob*, const GatherWG*, int, const Taps*, const KArgs&, int,
                                         double*, hipStream_t);

}  // namespace sbp
