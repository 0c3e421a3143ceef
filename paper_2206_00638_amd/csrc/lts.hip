// Local time stepping at 1:p for refined blocks: the vector kernels of the
// scheme (the operator itself is applied by the step kernels).
//
// The paper leaves multi-block coupling to later work and gives no local
// time stepping; the scheme is the explicit, energy-conserving local time
// stepping for second-order wave equations of Diaz and Grote, applied to the
// lossless leapfrog of Section V in its E-only form
//   E^{n+1} - 2 E^n + E^{n-1} = -dt^2 L E^n,   L = -A B,
// A = eps^-1 K_eh, B = mu^-1 K_he (E7-E12 with the SAT rows).  With P the
// projector onto the E nodes of the refined blocks and tau = dt / p, a coarse
// step is E^{n+1} = -E^{n-1} + 2 q_p with w = L (I - P) E^n, q_0 = E^n,
// q_1 = q_0 - tau^2/2 (w + L P q_0), q_{m+1} = 2 q_m - q_{m-1} - tau^2 (w + L P q_m).
//
// E^{n+1} differs from the leapfrog's (with H^{n+1/2} = H^{n-1/2} + dt B E^n,
// E^{n+1} = E^n + dt A H^{n+1/2}) only on E nodes within a cell of a refined
// block: L P reaches that far and no farther, and the refined rows of L read
// E no farther.  So a coarse step is the ordinary step of length dt on every
// block, followed by the recursion above on a near box (the refined blocks
// whole and the nodes of other blocks within two of their cells of a refined
// block), whose result replaces the ordinary step's there.  The H arrays
// keep the ordinary step's H, which the E-only scheme has no use for; away
// from the near boxes it is the leapfrog's.
//
// The operator is applied by one leapfrog step of unit time step on a
// scratch state holding E = u and H = 0: the H pass leaves B u, the E pass
// u + A B u = u - L u.  Those steps run on the tiles that meet a wider box
// (four cells), so that every H and E value the near box reads is formed
// from nonzero input; the scratch state is zero elsewhere.
#include <hip/hip_runtime.h>

#include "plan.h"

namespace sbp {

namespace {

// Whether node (i, j, k) of E component c exists (the node box pads every
// component to the largest extents).
__device__ __forceinline__ bool e_valid(const DevBlock& B, int c, int i, int j, int k) {
  const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
  if (c == 0) return i <= nx + 1 && j <= ny && k <= nz;
  if (c == 1) return i <= nx && j <= ny + 1 && k <= nz;
  return i <= nx && j <= ny && k <= nz + 1;
}

// Scratch state on the nodes of a tile list (one workgroup per tile;
// `threads` node columns x cz planes per tile):
//   mode 0: E = (I - P) E^n (the pool's E off the refined blocks);  H = 0
//   mode 1: E = P q (Q's E on the refined blocks; Q may be the pool);  H = 0
//   mode 2: E = 0;  H = the pool's H
template <typename T>
__global__ __launch_bounds__(256) void k_lts_prep(T* S, const T* pool, const T* Q, int mode, const Tile* tiles,
                                                 const DevBlock* blocks, const LtsBox* boxes, int threads, int cz) {
  const Tile tl = tiles[blockIdx.x];
  const DevBlock& B = blocks[tl.block];
  const int refined = boxes[tl.block].refined;
  const long long sx = B.sx, sxy = B.sxy, csz = B.csz;
  const long long plane = sx * (B.n[1] + 2);
  const int nz2 = B.n[2] + 2;
  for (int idx = threadIdx.x; idx < threads * cz; idx += blockDim.x) {
    const long long q = tl.q0 + idx % threads;
    const int k = tl.z0 + idx / threads;
    if (q >= plane || k >= nz2) continue;
    const int j = (int)(q / sx), i = (int)(q - j * sx);
    const long long o = B.foff + q + sxy * k;
    for (int c = 0; c < 3; ++c) {
      const long long e = o + c * csz, h = o + (3 + c) * csz;
      T v = T(0);
      if (e_valid(B, c, i, j, k)) {
        if (mode == 0 && !refined) v = pool[e];
        if (mode == 1 && refined) v = Q[e];
      }
      S[e] = v;
      S[h] = mode == 2 ? pool[h] : T(0);
    }
  }
}

// Element-wise steps over the near boxes (grid row y = block), E^n the
// pool's E, S = u - L u for the u of the preceding prep:
//   op 0: W = L (I - P) E^n = (I - P) E^n - S
//   op 1: first substep: Qo = E^n - tau2/2 (W + L P E^n), L P E^n = P E^n - S
//   op 2: later substep: Qo = 2 Qm - Qp - tau2 (W + L P Qm), L P Qm = P Qm - S
//         (Qp may be the pool, Qo may be Qp)
//   op 3: before the ordinary step: W = -Ep + 2 Qm (E^{n+1}); Ep = E^n
//   op 4: after it: E = W
//   op 5: Ep = E^n - coef S (E^{-1} = E^0 - dt A H^{-1/2}, S holding A H^{-1/2})
template <typename T>
__global__ __launch_bounds__(256) void k_lts_box(int op, T* pool, const T* S, T* W, const T* Qm, const T* Qp, T* Qo,
                                                T* Ep, double coef, const DevBlock* blocks, const LtsBox* boxes) {
  const DevBlock& B = blocks[blockIdx.y];
  const LtsBox bx = boxes[blockIdx.y];
  if (!bx.on) return;
  const int ex = bx.hi[0] - bx.lo[0] + 1, ey = bx.hi[1] - bx.lo[1] + 1, ez = bx.hi[2] - bx.lo[2] + 1;
  const long long per = (long long)ex * ey * ez;
  const T cf = (T)coef;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * per;
       t += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(t / per);
    long long r = t - c * per;
    const int kk = (int)(r / ((long long)ex * ey));
    r -= (long long)kk * ex * ey;
    const int jj = (int)(r / ex), ii = (int)(r - (long long)jj * ex);
    const int i = bx.lo[0] + ii, j = bx.lo[1] + jj, k = bx.lo[2] + kk;
    if (!e_valid(B, c, i, j, k)) continue;
    const long long e = B.foff + c * B.csz + i + B.sx * j + B.sxy * k;
    switch (op) {
      case 0: W[e] = (bx.refined ? T(0) : pool[e]) - S[e]; break;
      case 1: {
        const T en = pool[e];
        const T lpq = (bx.refined ? en : T(0)) - S[e];
        Qo[e] = en - (T(0.5) * cf) * (W[e] + lpq);
        break;
      }
      case 2: {
        const T qm = Qm[e];
        const T lpq = (bx.refined ? qm : T(0)) - S[e];
        Qo[e] = (T(2) * qm - Qp[e]) - cf * (W[e] + lpq);
        break;
      }
      case 3: {
        const T en = pool[e];
        W[e] = T(2) * Qm[e] - Ep[e];
        Ep[e] = en;
        break;
      }
      case 4: pool[e] = W[e]; break;
      default: Ep[e] = pool[e] - cf * S[e]; break;
    }
  }
}

// Whole E parts of every block (grid row y = block):
//   op 0: X = E (the pool)
//   op 1: X = E - dt S  (E^{-1} = E^0 - dt A H^{-1/2}, S holding A H^{-1/2})
//   op 2: energy W^{n+1/2} = sum M [(E^{n+1} - E^n)^2 + E^{n+1} (2 E^n - E^{n+1} - E^{n-1})] / (2 dt^2)
//         from X = E^{n-1}, Y = E^n, the pool = E^{n+1}: fp64 per workgroup
//         into partials[y * gridDim.x + x]
template <typename T>
__global__ __launch_bounds__(256) void k_lts_whole(int op, const T* pool, T* X, const T* Y, const T* S, double d,
                                                  const DevBlock* blocks, const void* mat_eps, double eps0,
                                                  double* partials) {
  __shared__ double red[4];
  const DevBlock& B = blocks[blockIdx.y];
  const long long csz = B.csz, sx = B.sx, sxy = B.sxy, plane = sx * (B.n[1] + 2);
  double acc = 0.0;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * csz;
       t += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(t / csz);
    const long long o = t - c * csz;
    const int k = (int)(o / sxy);
    const long long r = o - k * sxy;
    const int j = (int)(r / sx), i = (int)(r - j * sx);
    const long long e = B.foff + t;
    if (op == 0) {
      X[e] = pool[e];
    } else if (op == 1) {
      X[e] = pool[e] - (T)d * S[e];
    } else if (r < plane && e_valid(B, c, i, j, k)) {
      const NodeCells nc = node_cells_t<T>(B, mat_eps, c, i, j, k);
      const double mw = eps0 * (0.25 * nc.S) * e_weight(B, c, i, j, k);
      const double eo = (double)X[e], en = (double)Y[e], enew = (double)pool[e];
      const double df = enew - en;
      acc += mw * (df * df + enew * (2.0 * en - enew - eo));
    }
  }
  if (op != 2) return;
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[w];
    partials[blockIdx.y * gridDim.x + blockIdx.x] = d * sum;
  }
}

// Energy ring slot of a coarse step: the fixed-order sum of the partials
// (nparts > 0) or NaN (energy not formed at this step).
__global__ __launch_bounds__(256) void k_lts_store(const double* partials, int nparts, double* slot) {
  __shared__ double red[4];
  double s = 0.0;
  for (int p = threadIdx.x; p < nparts; p += blockDim.x) s += partials[p];
  s = wave_sum(s);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w];
    *slot = nparts > 0 ? tot : __builtin_nan("");
  }
}

}  // namespace

constexpr int kLtsGrid = 64;  // workgroups per block row of the box and whole-part kernels

template <typename T>
hipError_t lts_prep(void* S, const void* pool, const void* Q, int mode, const Tile* tiles, int ntiles,
                    const DevBlock* blocks, const LtsBox* boxes, int threads, int cz, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lts_prep<T>, dim3(ntiles), dim3(256), 0, s, (T*)S, (const T*)pool, (const T*)Q, mode, tiles,
                     blocks, boxes, threads, cz);
  return hipGetLastError();
}

template <typename T>
hipError_t lts_box(int op, int nblocks, void* pool, const void* S, void* W, const void* Qm, const void* Qp, void* Qo,
                   void* Ep, double coef, const DevBlock* blocks, const LtsBox* boxes, hipStream_t s) {
  hipLaunchKernelGGL(k_lts_box<T>, dim3(kLtsGrid, nblocks), dim3(256), 0, s, op, (T*)pool, (const T*)S, (T*)W,
                     (const T*)Qm, (const T*)Qp, (T*)Qo, (T*)Ep, coef, blocks, boxes);
  return hipGetLastError();
}

template <typename T>
hipError_t lts_whole(int op, int nblocks, const void* pool, void* X, const void* Y, const void* S, double d,
                     const DevBlock* blocks, const void* mat_eps, double eps0, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_lts_whole<T>, dim3(kLtsGrid, nblocks), dim3(256), 0, s, op, (const T*)pool, (T*)X,
                     (const T*)Y, (const T*)S, d, blocks, mat_eps, eps0, partials);
  return hipGetLastError();
}

hipError_t lts_store(const double* partials, int nparts, double* slot, hipStream_t s) {
  hipLaunchKernelGGL(k_lts_store, dim3(1), dim3(256), 0, s, partials, nparts, slot);
  return hipGetLastError();
}

#define SBP_LTS_INST(T)                                                                                             \
  template hipError_t lts_prep<T>(void*, const void*, const void*, int, const Tile*, int, const DevBlock*,           \
                                  const LtsBox*, int, int, hipStream_t);                                             \
  template hipError_t lts_box<T>(int, int, void*, const void*, void*, const void*, const void*, void*, void*, double, \
                                 const DevBlock*, const LtsBox*, hipStream_t);                                       \
  template hipError_t lts_whole<T>(int, int, const void*, void*, const void*, const void*, double, const DevBlock*, \
                                   const void*, double, double*, hipStream_t);
SBP_LTS_INST(float)
SBP_LTS_INST(double)
#undef SBP_LTS_INST

}  // namespace sbp
