// Kernels of the discrete adjoint of the leapfrog step (gradient of a region
// objective with respect to the per-cell relative permittivity).
//
// Objective: J = dt sum_{n=1..N} sum_{cells c in region} |Ebar_c^n|^2, with
// Ebar_c per component the mean of the four edges of cell c carrying it.
//
// For PEC/PMC faces and interfaces the SAT-modified difference operators are
// skew-adjoint in the norms of Section II (the energy identity behind E16):
// w_E . (C_e H) = -(w_H . C_h E), with C_e the E-update curl (D+ rows) and C_h
// the H-update curl (D- rows), w_E, w_H the products of the 1D norm weights.
// With that identity the adjoint recursion of the leapfrog step,
//   lam_H^{n+1/2} = lam_H^{n+3/2} + C_e^T (Cb lam_E^{n+1})
//   lam_E^n       = Ca lam_E^{n+1} + C_h^T (Db lam_H^{n+1/2}) + dJ/dE^n,
// becomes, for p = Cb lam_E / w_E and r = -Db lam_H / w_H, the forward step
// itself: r^{n+1/2} = r^{n+3/2} + Db C_h(p^{n+1}),
// p^n = Ca p^{n+1} + Cb (C_e(r^{n+1/2}) + dJ/dE^n / w_E).  The step kernels
// therefore run the adjoint on a second state; these kernels add the
// objective's source, accumulate dJ/dCb = sum_n lam_E^{n+1} (E^{n+1} - E^n)/Cb
// (lossless: Ca = 1; with lam_E = w_E p / Cb that is (w_E / Cb^2) sum_n
// p^{n+1} (E^{n+1} - E^n)), and chain dJ/dCb to the cells through Cb = 4 dt /
// (eps0 S), S the sum of the four (clamped) cells around the node.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "plan.h"

namespace sbp {

struct Region {
  int lo[3], hi[3];  // half-open cell box
};

namespace {

// Mean of component c (0 = Ex, 1 = Ey, 2 = Ez) over the four edges of cell
// (ci, cj, ck) that carry it: the "-" node of the cell centre along c, both
// "+" nodes of the cell along the other two axes.
template <typename T>
__device__ double cell_mean(const T* comp, const DevBlock& B, int c, int ci, int cj, int ck) {
  int node[3] = {ci, cj, ck};
  node[c] += 1;
  const int a1 = c == 0 ? 1 : 0, a2 = c == 2 ? 1 : 2;
  const long long st[3] = {1, B.sx, B.sxy};
  const long long o = node[0] + B.sx * node[1] + B.sxy * node[2];
  return 0.25 * (((double)comp[o] + (double)comp[o + st[a1]]) +
                 ((double)comp[o + st[a2]] + (double)comp[o + st[a1] + st[a2]]));
}

}  // namespace

// J += dt sum_{cells in region} |Ebar|^2 of the state in `pool` (one workgroup).
template <typename T>
__global__ __launch_bounds__(256) void k_adj_objective(const void* pool, const DevBlock* blocks, int block,
                                                      Region r, double dt, double* J) {
  __shared__ double red[4];
  const DevBlock& B = blocks[block];
  const T* base = (const T*)pool + B.foff;
  const int ex = r.hi[0] - r.lo[0], ey = r.hi[1] - r.lo[1], ez = r.hi[2] - r.lo[2];
  const int ncell = ex * ey * ez;
  double s = 0.0;
  for (int q = threadIdx.x; q < ncell; q += blockDim.x) {
    const int ci = r.lo[0] + q % ex, cj = r.lo[1] + (q / ex) % ey, ck = r.lo[2] + q / (ex * ey);
    for (int c = 0; c < 3; ++c) {
      const double m = cell_mean<T>(base + c * B.csz, B, c, ci, cj, ck);
      s += m * m;
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += red[w];
    J[0] += dt * t;
  }
}

// p += Cb / w_E * dJ/dE^n on the region's edge nodes; dJ/dE^n from the
// forward state E^n in `epool` (layout of the field pool).  `apool` is the
// adjoint state.  One thread per edge node of the region.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_source(void* apool, const void* epool, const DevBlock* blocks,
                                                   const void* mat_eps, int block, Region r, double dt) {
  const DevBlock& B = blocks[block];
  int cnt[3];
  int ext[3][3];
  for (int c = 0; c < 3; ++c) {
    int n = 1;
    for (int a = 0; a < 3; ++a) {
      ext[c][a] = (a == c) ? (r.hi[a] - r.lo[a]) : (r.hi[a] - r.lo[a] + 1);
      n *= ext[c][a];
    }
    cnt[c] = n;
  }
  const int total = cnt[0] + cnt[1] + cnt[2];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    int c = 0, q = t;
    while (q >= cnt[c]) q -= cnt[c++];
    int node[3];
    node[0] = q % ext[c][0];
    node[1] = (q / ext[c][0]) % ext[c][1];
    node[2] = q / (ext[c][0] * ext[c][1]);
    for (int a = 0; a < 3; ++a) node[a] += (a == c) ? r.lo[a] + 1 : r.lo[a];
    // cells of the region having this node as one of their four edges
    const T* e = (const T*)epool + B.foff + c * B.csz;
    double g = 0.0;
    int c0[3], c1[3];
    for (int a = 0; a < 3; ++a) {
      if (a == c) {
        c0[a] = c1[a] = node[a] - 1;
      } else {
        c0[a] = max(node[a] - 1, r.lo[a]);
        c1[a] = min(node[a], r.hi[a] - 1);
      }
    }
    for (int ck = c0[2]; ck <= c1[2]; ++ck)
      for (int cj = c0[1]; cj <= c1[1]; ++cj)
        for (int ci = c0[0]; ci <= c1[0]; ++ci) g += cell_mean<T>(e, B, c, ci, cj, ck);
    g *= 0.5 * dt;  // d/dE (dt Ebar^2) = 2 dt Ebar / 4 per cell
    const NodeCells nc = node_cells_t<T>(B, mat_eps, c, node[0], node[1], node[2]);
    const double cb = node_cb(B, nc.S);
    const long long o = node[0] + B.sx * node[1] + B.sxy * node[2];
    T* p = (T*)apool + B.foff + c * B.csz;
    p[o] = (T)((double)p[o] + cb / e_weight(B, c, node[0], node[1], node[2]) * g);
  }
}

// S += p^{n+1} (E^{n+1} - E^n) over the block's three E component arrays,
// flat (n = 3 x the component stride; nodes outside a component's grid are
// dropped in k_adj_node).  With w_E and Cb constant in time, dJ/dCb of the
// node is (w_E / Cb^2) S after the sweep; k_adj_node applies the factor.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_grad(const T* __restrict__ p, const T* __restrict__ enew,
                                                 const T* __restrict__ eold, long long n, double* __restrict__ S) {
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
    S[t] += (double)p[t] * ((double)enew[t] - (double)eold[t]);
}

// dJ/d eps_r per cell: the sum over the E nodes of dJ/dCb * dCb/d eps_r(cell),
// with dJ/dCb = (w_E / Cb^2) S from k_adj_grad's sums and dCb/d eps_r =
// -Cb / S_eps for each occurrence of the cell among the node's four.  Two
// passes, no atomics, so the result does not depend on the order in which
// workgroups run: k_adj_node turns each E node's S in place into its
// contribution per occurrence, d = -(w_E S / Cb) / S_eps; k_adj_cells then
// sums, for each cell, the contributions of the E nodes around it in a fixed
// order, each as often as the cell occurs in the node's (clamped) four.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_node(const DevBlock* blocks, const void* mat_eps, int block, double* G) {
  const DevBlock& B = blocks[block];
  const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
  const long long sx = B.sx, sxy = B.sxy;
  const long long plane = sx * (ny + 2);
  const long long nodes = plane * (nz + 2);
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * nodes;
       t += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(t / nodes);
    const long long q = t - c * nodes;
    const int k = (int)(q / plane);
    const long long rr = q - k * plane;
    const int j = (int)(rr / sx), i = (int)(rr - j * sx);
    const bool valid = c == 0 ? (j <= ny && k <= nz) : (c == 1 ? (i <= nx && k <= nz) : (i <= nx && j <= ny));
    const long long o = i + sx * j + sxy * k;
    double& g = G[c * B.csz + o];
    if (!valid || g == 0.0) {
      g = 0.0;
      continue;
    }
    const NodeCells nc = node_cells_t<T>(B, mat_eps, c, i, j, k);
    const double cb = node_cb(B, nc.S);
    g = -(e_weight(B, c, i, j, k) * g / cb) / nc.S;
  }
}

// Along one axis: the node indices whose cell list holds cell `cc`, and how
// often.  "-" grid (the component's own axis): node r lies in cell
// clamp(r - 1), so r = cc + 1, and also 0 for the first cell and n + 1 for
// the last.  "+" grid: node r lies in cells clamp(r - 1) and clamp(r), so
// r = cc (twice for the first cell) and r = cc + 1 (twice for the last).
__device__ __forceinline__ int axis_nodes(bool minus, int n, int cc, int r[3], int m[3]) {
  if (minus) {
    int q = 0;
    r[q] = cc + 1;
    m[q++] = 1;
    if (cc == 0) { r[q] = 0; m[q++] = 1; }
    if (cc == n - 1) { r[q] = n + 1; m[q++] = 1; }
    return q;
  }
  r[0] = cc;
  m[0] = cc == 0 ? 2 : 1;
  r[1] = cc + 1;
  m[1] = cc == n - 1 ? 2 : 1;
  return 2;
}

__global__ __launch_bounds__(256) void k_adj_cells(const DevBlock* blocks, int block, const double* G, double* grad) {
  const DevBlock& B = blocks[block];
  const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
  const long long ncell = (long long)nx * ny * nz;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
       t += (long long)gridDim.x * blockDim.x) {
    const int ci = (int)(t % nx), cj = (int)((t / nx) % ny), ck = (int)(t / ((long long)nx * ny));
    double acc = 0.0;
    for (int c = 0; c < 3; ++c) {
      int rx[3], mx[3], ry[3], my[3], rz[3], mz[3];
      const int qx = axis_nodes(c == 0, nx, ci, rx, mx);
      const int qy = axis_nodes(c == 1, ny, cj, ry, my);
      const int qz = axis_nodes(c == 2, nz, ck, rz, mz);
      const double* gc = G + c * B.csz;
      for (int a = 0; a < qz; ++a)
        for (int b = 0; b < qy; ++b)
          for (int d = 0; d < qx; ++d)
            acc += (double)(mx[d] * my[b] * mz[a]) * gc[rx[d] + B.sx * ry[b] + B.sxy * rz[a]];
    }
    grad[t] = acc;
  }
}

template <typename T>
hipError_t launch_adj_objective(const void* pool, const DevBlock* blocks, int block, const int r[6], double dt,
                                double* J, hipStream_t s) {
  Region R{{r[0], r[2], r[4]}, {r[1], r[3], r[5]}};
  hipLaunchKernelGGL(k_adj_objective<T>, dim3(1), dim3(256), 0, s, pool, blocks, block, R, dt, J);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_adj_source(void* apool, const void* epool, const DevBlock* blocks, const void* mat_eps, int block,
                             const int r[6], double dt, hipStream_t s) {
  Region R{{r[0], r[2], r[4]}, {r[1], r[3], r[5]}};
  long long total = 0;
  for (int c = 0; c < 3; ++c) {
    long long n = 1;
    for (int a = 0; a < 3; ++a) n *= (a == c) ? (R.hi[a] - R.lo[a]) : (R.hi[a] - R.lo[a] + 1);
    total += n;
  }
  const int grid = (int)std::min<long long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_adj_source<T>, dim3(grid), dim3(256), 0, s, apool, epool, blocks, mat_eps, block, R, dt);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_adj_grad(const void* p, const void* enew, const void* eold, long long n, double* S,
                           hipStream_t s) {
  const int grid = (int)std::min<long long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_adj_grad<T>, dim3(grid), dim3(256), 0, s, (const T*)p, (const T*)enew, (const T*)eold, n, S);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_adj_cells(const DevBlock* blocks, const void* mat_eps, int block, double* G, double* grad,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_adj_node<T>, dim3(4096), dim3(256), 0, s, blocks, mat_eps, block, G);
  hipLaunchKernelGGL(k_adj_cells, dim3(4096), dim3(256), 0, s, blocks, block, (const double*)G, grad);
  return hipGetLastError();
}

template hipError_t launch_adj_objective<float>(const void*, const DevBlock*, int, const int*, double, double*,
                                                hipStream_t);
template hipError_t launch_adj_objective<double>(const void*, const DevBlock*, int, const int*, double, double*,
                                                 hipStream_t);
template hipError_t launch_adj_source<float>(void*, const void*, const DevBlock*, const void*, int, const int*,
                                             double, hipStream_t);
template hipError_t launch_adj_source<double>(void*, const void*, const DevBlock*, const void*, int, const int*,
                                              double, hipStream_t);
template hipError_t launch_adj_grad<float>(const void*, const void*, const void*, long long, double*, hipStream_t);
template hipError_t launch_adj_grad<double>(const void*, const void*, const void*, long long, double*, hipStream_t);
template hipError_t launch_adj_cells<float>(const DevBlock*, const void*, int, double*, double*, hipStream_t);
template hipError_t launch_adj_cells<double>(const DevBlock*, const void*, int, double*, double*, hipStream_t);

}  // namespace sbp
