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
// E no farther.  So a coarse step is the ordinary step of length dt on the
// blocks that are not refined, followed by the recursion above, in its own
// order of operations, on a near box (the refined blocks whole and the nodes
// of other blocks within two of their cells of a refined block), whose
// result replaces the ordinary step's there.  The H arrays keep the ordinary
// step's H, which the E-only scheme has no use for; away from the near boxes
// it is the leapfrog's; on the refined blocks it is not stepped.
//
// The operator is applied by one leapfrog step of unit time step on a
// scratch state holding E = u and H = 0: the H pass leaves B u, the E pass
// u + A B u = u - L u.  Those steps run on the tiles that meet a wider box
// (four cells), so that every H and E value the near box reads is formed
// from nonzero input; the scratch state is zero elsewhere.  The element-wise
// parts of the recursion run over the same tiles, each fused with the
// preparation of the next scratch state.
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

__device__ __forceinline__ bool in_box(const LtsBox& x, int i, int j, int k) {
  return x.on && i >= x.lo[0] && i <= x.hi[0] && j >= x.lo[1] && j <= x.hi[1] && k >= x.lo[2] && k <= x.hi[2];
}

// One phase of a coarse step on the nodes of a tile list (one workgroup per
// tile; `threads` node columns x cz planes per tile).  E^n is the pool's E
// (until the ordinary step), S = u - L u for the u of the preceding scratch
// state.  First, on the E nodes of the near boxes:
//   op 0 (u = (I - P) E^n): W = L (I - P) E^n = (I - P) E^n - S
//   op 1 (u = P E^n): q_1 = E^n - tau2/2 (W + L P E^n), L P E^n = P E^n - S;
//        into Qo
//   op 2 (u = P q_m): q_{m+1} = 2 Qm - Qp - tau2 (W + L P q_m),
//        L P q_m = P q_m - S (Qp = q_{m-1}, the pool for m = 1); into Qo, or
//        with `last`: W = E^{n+1} = 2 q_{m+1} - Ep and Ep = E^n
//   op 3: the pool's E = W (after the ordinary step)
//   op 4: Ep = E^n - dt S (E^{-1}, S holding A H^{-1/2})
// Then the next scratch state on every node of the tiles (nmode):
//   0: E = (I - P) E (the pool's);  1: E = P q, q = E^n after op 0, the q
//   just formed after ops 1 and 2;  2: E = 0, H = the pool's H;
//   H = 0 in modes 0 and 1.
template <typename T>
__global__ __launch_bounds__(256) void k_lts_phase(int op, int nmode, int last, T* pool, T* S, T* W, const T* Qm,
                                                  const T* Qp, T* Qo, T* Ep, double tau2, double dt,
                                                  const Tile* tiles, const DevBlock* blocks, const LtsBox* boxes,
                                                  int threads, int cz) {
  const Tile tl = tiles[blockIdx.x];
  const DevBlock& B = blocks[tl.block];
  const LtsBox bx = boxes[tl.block];
  const long long sxy = B.sxy, csz = B.csz;
  const int sx = (int)B.sx, plane = sx * (B.n[1] + 2);
  const int nz2 = B.n[2] + 2;
  const T t2 = (T)tau2, tdt = (T)dt;
  for (int idx = threadIdx.x; idx < threads * cz; idx += blockDim.x) {
    const int q = tl.q0 + idx % threads;
    const int k = tl.z0 + idx / threads;
    if (q >= plane || k >= nz2) continue;
    const int j = q / sx, i = q - j * sx;
    const long long o = B.foff + q + sxy * k;
    const bool near = in_box(bx, i, j, k);
    for (int c = 0; c < 3; ++c) {
      const long long e = o + c * csz, h = o + (3 + c) * csz;
      const bool valid = e_valid(B, c, i, j, k);
      T qnext = T(0);
      if (valid && near) {
        if (op == 0) {
          const T en = pool[e];
          W[e] = (bx.refined ? T(0) : en) - S[e];
          qnext = en;
        } else if (op == 1) {
          const T en = pool[e];
          const T lpq = (bx.refined ? en : T(0)) - S[e];
          const T q1 = en - (T(0.5) * t2) * (W[e] + lpq);
          Qo[e] = q1;
          qnext = q1;
        } else if (op == 2) {
          const T qm = Qm[e];
          const T lpq = (bx.refined ? qm : T(0)) - S[e];
          const T qn = (T(2) * qm - Qp[e]) - t2 * (W[e] + lpq);
          if (last) {
            const T en = pool[e];
            W[e] = T(2) * qn - Ep[e];
            Ep[e] = en;
          } else {
            Qo[e] = qn;
            qnext = qn;
          }
        } else if (op == 3) {
          pool[e] = W[e];
        } else if (op == 4) {
          Ep[e] = pool[e] - tdt * S[e];
        }
      }
      if (nmode >= 0) {
        T v = T(0);
        if (valid) {
          if (nmode == 0 && !bx.refined) v = pool[e];
          if (nmode == 1 && bx.refined) v = qnext;
        }
        S[e] = v;
        S[h] = nmode == 2 ? pool[h] : T(0);
      }
    }
  }
}

// Whole E parts of every block (grid row y = block):
//   op 0: X = E (the pool)
//   op 1: X = E - dt S  (E^{-1} = E^0 - dt A H^{-1/2}, S holding A H^{-1/2})
template <typename T>
__global__ __launch_bounds__(256) void k_lts_whole(int op, const T* pool, T* X, const T* S, double d,
                                                  const DevBlock* blocks) {
  const DevBlock& B = blocks[blockIdx.y];
  const T dd = (T)d;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * B.csz;
       t += (long long)gridDim.x * blockDim.x) {
    const long long e = B.foff + t;
    X[e] = op == 0 ? pool[e] : pool[e] - dd * S[e];
  }
}

// The energy W^{n+1/2} = sum M [(E^{n+1} - E^n)^2 + E^{n+1} (2 E^n - E^{n+1} - E^{n-1})] / (2 dt^2)
// (M the E16 weights times eps) from X = E^{n-1}, Y = E^n and the pool's
// E^{n+1}, over the nodes of a tile list (one workgroup per tile): fp64 per
// workgroup into partials[blockIdx.x], times `scale`.
template <typename T>
__global__ __launch_bounds__(256) void k_lts_energy(const T* pool, const T* X, const T* Y, double scale,
                                                   const Tile* tiles, const DevBlock* blocks, const void* mat_eps,
                                                   double eps0, int threads, int cz, double* partials) {
  __shared__ double red[4];
  const Tile tl = tiles[blockIdx.x];
  const DevBlock& B = blocks[tl.block];
  const long long sxy = B.sxy, csz = B.csz;
  const int sx = (int)B.sx, plane = sx * (B.n[1] + 2);
  const int nz2 = B.n[2] + 2;
  double acc = 0.0;
  for (int idx = threadIdx.x; idx < threads * cz; idx += blockDim.x) {
    const int q = tl.q0 + idx % threads;
    const int k = tl.z0 + idx / threads;
    if (q >= plane || k >= nz2) continue;
    const int j = q / sx, i = q - j * sx;
    const long long o = B.foff + q + sxy * k;
    for (int c = 0; c < 3; ++c) {
      if (!e_valid(B, c, i, j, k)) continue;
      const long long e = o + c * csz;
      const NodeCells nc = node_cells_t<T>(B, mat_eps, c, i, j, k);
      const double mw = eps0 * (0.25 * nc.S) * e_weight(B, c, i, j, k);
      const double eo = (double)X[e], en = (double)Y[e], enew = (double)pool[e];
      const double df = enew - en;
      acc += mw * (df * df + enew * (2.0 * en - enew - eo));
    }
  }
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[w];
    partials[blockIdx.x] = scale * sum;
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

constexpr int kLtsGrid = 512;  // workgroups per block row of the copy kernel

template <typename T>
hipError_t lts_phase(int op, int nmode, int last, void* pool, void* S, void* Y, const void* Qm, const void* Qp,
                     void* Qo, void* Ep, double tau2, double dt, const Tile* tiles, int ntiles, const DevBlock* blocks,
                     const LtsBox* boxes, int threads, int cz, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lts_phase<T>, dim3(ntiles), dim3(256), 0, s, op, nmode, last, (T*)pool, (T*)S, (T*)Y,
                     (const T*)Qm, (const T*)Qp, (T*)Qo, (T*)Ep, tau2, dt, tiles, blocks, boxes, threads, cz);
  return hipGetLastError();
}

template <typename T>
hipError_t lts_whole(int op, int nblocks, const void* pool, void* X, const void* S, double d, const DevBlock* blocks,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_lts_whole<T>, dim3(kLtsGrid, nblocks), dim3(256), 0, s, op, (const T*)pool, (T*)X,
                     (const T*)S, d, blocks);
  return hipGetLastError();
}

template <typename T>
hipError_t lts_energy(const void* pool, const void* X, const void* Y, double scale, const Tile* tiles, int ntiles,
                      const DevBlock* blocks, const void* mat_eps, double eps0, int threads, int cz, double* partials,
                      hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lts_energy<T>, dim3(ntiles), dim3(256), 0, s, (const T*)pool, (const T*)X, (const T*)Y, scale,
                     tiles, blocks, mat_eps, eps0, threads, cz, partials);
  return hipGetLastError();
}

hipError_t lts_store(const double* partials, int nparts, double* slot, hipStream_t s) {
  hipLaunchKernelGGL(k_lts_store, dim3(1), dim3(256), 0, s, partials, nparts, slot);
  return hipGetLastError();
}

#define SBP_LTS_INST(T)                                                                                             \
  template hipError_t lts_phase<T>(int, int, int, void*, void*, void*, const void*, const void*, void*, void*,       \
                                   double, double, const Tile*, int, const DevBlock*, const LtsBox*, int, int,       \
                                   hipStream_t);                                                                     \
  template hipError_t lts_whole<T>(int, int, const void*, void*, const void*, double, const DevBlock*, hipStream_t); \
  template hipError_t lts_energy<T>(const void*, const void*, const void*, double, const Tile*, int, const DevBlock*, \
                                    const void*, double, int, int, double*, hipStream_t);
SBP_LTS_INST(float)
SBP_LTS_INST(double)
#undef SBP_LTS_INST

}  // namespace sbp
