// Leapfrog step kernels of the 3D SBP-SAT FDTD method for gfx950.
//
// Memory-bound staggered stencil: one thread per (i, j) node column of a
// tile, marching through the tile's z planes so that the z-neighbour of the
// previous plane stays in registers; x/y neighbours come from the wave's own
// loads through the L1/L2.  Interior rows are the two-point Yee difference
// (Section II-A: the interior nodes are Yee's); rows within two (D+) or three
// (D-) nodes of a block face take the Appendix closure rows with the SAT row
// changes folded in (PEC in the H update, PMC / absorbing in the E update,
// interface rows reading gathered neighbour values).  Every node update is a
// pure function of the previous fields, so results do not depend on the
// tile shape or on how tiles map to workgroups.
//
// The discrete energy W^n (E16 with the leapfrog pairing of H) is reduced in
// fp64 per workgroup and finished by the last workgroup of each launch.

#include "plan.h"

namespace sbp {


__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Norm weight (diagonal of P+ or P- with h) of node r on an axis of n cells.
__device__ __forceinline__ double wplus(int n, int r, double h) {
  return (r == 0 || r == n) ? 0.5 * h : h;
}
__device__ __forceinline__ double wminus(int n, int r, double h) {
  if (r == 0 || r == n + 1) return 0.5 * h;
  if (r == 1 || r == n) return 0.25 * h;
  if (r == 2 || r == n - 1) return 1.25 * h;
  return h;
}

__device__ __forceinline__ double face_value(const KArgs& a, const DevBlock& B, int face, int is_h,
                                             int slot, int i, int j, int k) {
  const int axis = face >> 1;
  const long long t = axis == 0 ? (long long)j + (long long)(B.n[1] + 2) * k
                    : axis == 1 ? (long long)i + (long long)(B.n[0] + 2) * k
                                : (long long)i + (long long)(B.n[0] + 2) * j;
  return a.face[B.fboff[face] + (long long)(is_h * 2 + slot) * B.fsz[face] + t];
}

// D- row r along `axis` applied to u at node offset o (the node with index r
// on that axis), times 1/h.  Closure rows come from the block's table.
template <typename T>
__device__ __forceinline__ double dminus(const KArgs& a, const DevBlock& B, int axis, const T* u,
                                         long long o, long long st, int r, int slot, int i, int j,
                                         int k) {
  const int n = B.n[axis];
  if (r >= 3 && r <= n - 2) return ((double)u[o] - (double)u[o - st]) * B.ih[axis];
  const int ci = r < 3 ? r : r - (n - 1) + 3;
  const Row& R = B.dm[axis][ci];
  const T* p = u + o + (long long)R.s * st;
  double v = R.c[0] * (double)p[0] + R.c[1] * (double)p[st] + R.c[2] * (double)p[2 * st];
  if (R.nbr) v += R.cn * face_value(a, B, 2 * axis + (r >= 3 ? 1 : 0), 0, slot, i, j, k);
  return v;
}

// D+ row r along `axis`, times 1/h.
template <typename T>
__device__ __forceinline__ double dplus(const KArgs& a, const DevBlock& B, int axis, const T* u,
                                        long long o, long long st, int r, int slot, int i, int j,
                                        int k) {
  const int n = B.n[axis];
  if (r >= 2 && r <= n - 2) return ((double)u[o + st] - (double)u[o]) * B.ih[axis];
  const int ci = r < 2 ? r : r - (n - 1) + 2;
  const Row& R = B.dp[axis][ci];
  const T* p = u + o + (long long)R.s * st;
  double v = R.c[0] * (double)p[0] + R.c[1] * (double)p[st] + R.c[2] * (double)p[2 * st];
  if (R.nbr) v += R.cn * face_value(a, B, 2 * axis + (r >= 2 ? 1 : 0), 1, slot, i, j, k);
  return v;
}

template <typename T>
__device__ __forceinline__ T cell(const void* arr, long long coff, const DevBlock& B, int ci, int cj,
                                  int ck) {
  return ((const T*)arr)[coff + ci + (long long)B.n[0] * (cj + (long long)B.n[1] * ck)];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ double load_coherent(const double* p) {
  unsigned long long b = __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)b);
}

// Reduces `v` over the launch.  The last workgroup to finish writes (E
// update: slot n+1 = sum) or adds (H update: slot n += sum) the total, flags
// a non-finite energy, resets the counter and, for the E update, advances
// the step index.
__device__ void finish_energy(double v, const KArgs& a, long long nstep, bool e_mode) {
  __shared__ double red[16];
  __shared__ int last;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    a.partials[blockIdx.x] = s;
    __threadfence();
    const unsigned prev = atomicAdd(&a.st->counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double s = 0.0;
  for (int p = threadIdx.x; p < (int)gridDim.x; p += blockDim.x) s += load_coherent(a.partials + p);
  s = wave_sum(s);
  __syncthreads();
  if (lane == 0) red[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int w = 0; w < nw; ++w) tot += red[w];
    if (e_mode) {
      const int slot = (int)((nstep + 1) % a.ecap);
      a.energy[slot] = tot;
    } else {
      const int slot = (int)(nstep % a.ecap);
      tot += a.energy[slot];
      a.energy[slot] = tot;
    }
    if (!isfinite(tot)) a.st->flags |= 1;
    a.st->counter = 0;
    if (e_mode) a.st->step = nstep + 1;
  }
}

// ---------------------------------------------------------------- H update
// H^{n+1/2} = H^{n-1/2} + dt/mu * (E10-E12 with the PEC/interface rows),
// plus the H part of W^n: 1/2 mu w H^{n+1/2} H^{n-1/2}.
template <typename T>
__global__ __launch_bounds__(512) void k_h_update(KArgs a) {
  double eacc = 0.0;
  const long long nstep = a.st->step;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile tl = a.tiles[t];
    const DevBlock& B = a.blocks[tl.block];
    const int i = tl.x0 + (int)threadIdx.x % a.tx;
    const int j = tl.y0 + (int)threadIdx.x / a.tx;
    const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
    if (i > nx + 1 || j > ny + 1) continue;
    const int k0 = tl.z0, k1 = min(tl.z0 + a.cz, nz + 2);
    const long long sx = B.sx, sxy = B.sxy;
    T* base = (T*)a.pool + B.foff;
    const T* Ex = base;
    const T* Ey = base + B.csz;
    const T* Ez = base + 2 * B.csz;
    T* Hx = base + 3 * B.csz;
    T* Hy = base + 4 * B.csz;
    T* Hz = base + 5 * B.csz;
    const double mu_u = a.mu0 * B.mu_r0;
    const bool xin = i >= 3 && i <= nx - 2, yin = j >= 3 && j <= ny - 2;
    const bool has_mu = B.mat & MAT_MU;
    // probes of this column (H components)
    int pk[2] = {-1, -1}, pc[2] = {0, 0}, pid[2] = {0, 0};
    {
      int q = 0;
      for (int p = 0; p < B.nprb && q < 2; ++p) {
        const Probe& P = a.prb[B.prb0 + p];
        if (P.comp >= HX && P.i == i && P.j == j && P.k >= k0 && P.k < k1) {
          pk[q] = P.k; pc[q] = P.comp; pid[q] = B.prb0 + p; ++q;
        }
      }
    }
    const double wxp = wplus(nx, i, B.h[0]), wxm = wminus(nx, i, B.h[0]);
    const double wyp = wplus(ny, j, B.h[1]), wym = wminus(ny, j, B.h[1]);
    const int ci0 = clampi(i - 1, 0, nx - 1), ci1 = clampi(i, 0, nx - 1);
    const int cj0 = clampi(j - 1, 0, ny - 1);
    const int cj1 = clampi(j, 0, ny - 1);
    long long o = i + sx * j + sxy * k0;
    T exm = T(0), eym = T(0);
    if (k0 > 0) { exm = Ex[o - sxy]; eym = Ey[o - sxy]; }
    for (int k = k0; k < k1; ++k, o += sxy) {
      const T ex = Ex[o], ey = Ey[o], ez = Ez[o];
      const T hx = Hx[o], hy = Hy[o], hz = Hz[o];
      const bool zin = k >= 3 && k <= nz - 2;
      // node permeability: mean over the (two) cells containing the H node
      double mux = mu_u, muy = mu_u, muz = mu_u;
      if (has_mu) {
        const int ck0 = clampi(k - 1, 0, nz - 1), ck1 = clampi(k, 0, nz - 1);
        const double A0 = (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj0, ck0);
        const double B0 = (double)cell<T>(a.mat_mu, B.coff, B, ci1, cj0, ck0);
        const double C0 = (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj1, ck0);
        const double A1 = (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj0, ck1);
        mux = a.mu0 * (0.5 * (A0 + B0));
        muy = a.mu0 * (0.5 * (A0 + C0));
        muz = a.mu0 * (0.5 * (A0 + A1));
      }
      const double dbx = a.dt / mux, dby = a.dt / muy, dbz = a.dt / muz;
      T nhx = hx, nhy = hy, nhz = hz;
      if (xin && yin && zin) {
        const T ez_im = Ez[o - 1], ey_im = Ey[o - 1];
        const T ez_jm = Ez[o - sx], ex_jm = Ex[o - sx];
        nhx = hx + (T)dbx * ((ey - eym) * (T)B.ih[2] - (ez - ez_jm) * (T)B.ih[1]);
        nhy = hy + (T)dby * ((ez - ez_im) * (T)B.ih[0] - (ex - exm) * (T)B.ih[2]);
        nhz = hz + (T)dbz * ((ex - ex_jm) * (T)B.ih[1] - (ey - ey_im) * (T)B.ih[0]);
      } else {
        if (i <= nx) {  // Hx (x+, y-, z-): dz Ey - dy Ez
          const double d = dminus<T>(a, B, 2, Ey, o, sxy, k, 1, i, j, k) -
                           dminus<T>(a, B, 1, Ez, o, sx, j, 1, i, j, k);
          nhx = (T)((double)hx + dbx * d);
        }
        if (j <= ny) {  // Hy (x-, y+, z-): dx Ez - dz Ex
          const double d = dminus<T>(a, B, 0, Ez, o, 1, i, 1, i, j, k) -
                           dminus<T>(a, B, 2, Ex, o, sxy, k, 0, i, j, k);
          nhy = (T)((double)hy + dby * d);
        }
        if (k <= nz) {  // Hz (x-, y-, z+): dy Ex - dx Ey
          const double d = dminus<T>(a, B, 1, Ex, o, sx, j, 0, i, j, k) -
                           dminus<T>(a, B, 0, Ey, o, 1, i, 0, i, j, k);
          nhz = (T)((double)hz + dbz * d);
        }
      }
      const double wzp = wplus(nz, k, B.h[2]), wzm = wminus(nz, k, B.h[2]);
      if (i <= nx) {
        Hx[o] = nhx;
        eacc += 0.5 * mux * wxp * wym * wzm * (double)nhx * (double)hx;
      }
      if (j <= ny) {
        Hy[o] = nhy;
        eacc += 0.5 * muy * wxm * wyp * wzm * (double)nhy * (double)hy;
      }
      if (k <= nz) {
        Hz[o] = nhz;
        eacc += 0.5 * muz * wxm * wym * wzp * (double)nhz * (double)hz;
      }
      for (int q = 0; q < 2; ++q)
        if (pk[q] == k) {
          const T v = pc[q] == HX ? nhx : (pc[q] == HY ? nhy : nhz);
          a.probes[(long long)pid[q] * a.pcap + nstep % a.pcap] = (double)v;
        }
      exm = ex;
      eym = ey;
    }
  }
  finish_energy(eacc, a, nstep, false);
}

__device__ __forceinline__ double waveform(const Source& s, double t) {
  const double d = t - s.t0;
  const double g = exp(-4.0 * M_PI * d * d / (s.tw * s.tw));
  return s.wave == 1 ? sin(2.0 * M_PI * s.f0 * t) * g : g;
}

// ---------------------------------------------------------------- E update
// E^{n+1} = Ca E^n + Cb (E7-E9 with the PMC/absorbing/interface rows + J),
// plus the E part of W^{n+1}: 1/2 eps w (E^{n+1})^2.
template <typename T>
__global__ __launch_bounds__(512) void k_e_update(KArgs a) {
  double eacc = 0.0;
  const long long nstep = a.st->step;
  const double tsrc = ((double)nstep + 0.5) * a.dt;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile tl = a.tiles[t];
    const DevBlock& B = a.blocks[tl.block];
    const int i = tl.x0 + (int)threadIdx.x % a.tx;
    const int j = tl.y0 + (int)threadIdx.x / a.tx;
    const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
    if (i > nx + 1 || j > ny + 1) continue;
    const int k0 = tl.z0, k1 = min(tl.z0 + a.cz, nz + 2);
    const long long sx = B.sx, sxy = B.sxy;
    T* base = (T*)a.pool + B.foff;
    T* Ex = base;
    T* Ey = base + B.csz;
    T* Ez = base + 2 * B.csz;
    const T* Hx = base + 3 * B.csz;
    const T* Hy = base + 4 * B.csz;
    const T* Hz = base + 5 * B.csz;
    const bool xin = i >= 2 && i <= nx - 2, yin = j >= 2 && j <= ny - 2;
    const bool has_eps = B.mat & MAT_EPS, has_sig = B.mat & MAT_SIG;
    // sources and probes of this column
    int sk[2] = {-1, -1}, sc[2] = {0, 0};
    double sv[2] = {0.0, 0.0};
    int pk[2] = {-1, -1}, pc[2] = {0, 0}, pid[2] = {0, 0};
    {
      int q = 0;
      for (int s = 0; s < B.nsrc && q < 2; ++s) {
        const Source& S = a.src[B.src0 + s];
        if (S.i == i && S.j == j && S.k >= k0 && S.k < k1) {
          sk[q] = S.k; sc[q] = S.comp; sv[q] = S.amp * waveform(S, tsrc); ++q;
        }
      }
      q = 0;
      for (int p = 0; p < B.nprb && q < 2; ++p) {
        const Probe& P = a.prb[B.prb0 + p];
        if (P.comp < HX && P.i == i && P.j == j && P.k >= k0 && P.k < k1) {
          pk[q] = P.k; pc[q] = P.comp; pid[q] = B.prb0 + p; ++q;
        }
      }
    }
    const double wxp = wplus(nx, i, B.h[0]), wxm = wminus(nx, i, B.h[0]);
    const double wyp = wplus(ny, j, B.h[1]), wym = wminus(ny, j, B.h[1]);
    const int ci0 = clampi(i - 1, 0, nx - 1), ci1 = clampi(i, 0, nx - 1);
    const int cj0 = clampi(j - 1, 0, ny - 1), cj1 = clampi(j, 0, ny - 1);
    // per-cell permittivity / conductivity of the 2x2 cell columns around (i, j)
    double eA0 = B.eps_r0, eB0 = B.eps_r0, eC0 = B.eps_r0, eD0 = B.eps_r0;
    double sA0 = B.sig0, sB0 = B.sig0, sC0 = B.sig0, sD0 = B.sig0;
    {
      const int ck = clampi(k0 - 1, 0, nz - 1);
      if (has_eps) {
        eA0 = (double)cell<T>(a.mat_eps, B.coff, B, ci0, cj0, ck);
        eB0 = (double)cell<T>(a.mat_eps, B.coff, B, ci1, cj0, ck);
        eC0 = (double)cell<T>(a.mat_eps, B.coff, B, ci0, cj1, ck);
        eD0 = (double)cell<T>(a.mat_eps, B.coff, B, ci1, cj1, ck);
      }
      if (has_sig) {
        sA0 = (double)cell<T>(a.mat_sig, B.coff, B, ci0, cj0, ck);
        sB0 = (double)cell<T>(a.mat_sig, B.coff, B, ci1, cj0, ck);
        sC0 = (double)cell<T>(a.mat_sig, B.coff, B, ci0, cj1, ck);
        sD0 = (double)cell<T>(a.mat_sig, B.coff, B, ci1, cj1, ck);
      }
    }
    long long o = i + sx * j + sxy * k0;
    T hx = Hx[o], hy = Hy[o];
    for (int k = k0; k < k1; ++k, o += sxy) {
      const int ck = clampi(k, 0, nz - 1);
      double eA1 = B.eps_r0, eB1 = B.eps_r0, eC1 = B.eps_r0, eD1 = B.eps_r0;
      double sA1 = B.sig0, sB1 = B.sig0, sC1 = B.sig0, sD1 = B.sig0;
      if (has_eps) {
        eA1 = (double)cell<T>(a.mat_eps, B.coff, B, ci0, cj0, ck);
        eB1 = (double)cell<T>(a.mat_eps, B.coff, B, ci1, cj0, ck);
        eC1 = (double)cell<T>(a.mat_eps, B.coff, B, ci0, cj1, ck);
        eD1 = (double)cell<T>(a.mat_eps, B.coff, B, ci1, cj1, ck);
      }
      if (has_sig) {
        sA1 = (double)cell<T>(a.mat_sig, B.coff, B, ci0, cj0, ck);
        sB1 = (double)cell<T>(a.mat_sig, B.coff, B, ci1, cj0, ck);
        sC1 = (double)cell<T>(a.mat_sig, B.coff, B, ci0, cj1, ck);
        sD1 = (double)cell<T>(a.mat_sig, B.coff, B, ci1, cj1, ck);
      }
      // node means over the containing cells
      const double epx = a.eps0 * (0.25 * ((eA0 + eC0) + (eA1 + eC1)));
      const double epy = a.eps0 * (0.25 * ((eA0 + eB0) + (eA1 + eB1)));
      const double epz = a.eps0 * (0.25 * ((eA0 + eB0) + (eC0 + eD0)));
      double sgx = 0.25 * ((sA0 + sC0) + (sA1 + sC1));
      double sgy = 0.25 * ((sA0 + sB0) + (sA1 + sB1));
      double sgz = 0.25 * ((sA0 + sB0) + (sC0 + sD0));
      const T ex = Ex[o], ey = Ey[o], ez = Ez[o];
      const T hz = Hz[o];
      const bool zin = k >= 2 && k <= nz - 2;
      const T hxn = (k + 1 < nz + 2) ? Hx[o + sxy] : T(0);
      const T hyn = (k + 1 < nz + 2) ? Hy[o + sxy] : T(0);
      double cx, cy, cz;  // curl terms (E7-E9), already / h
      bool fast = xin && yin && zin;
      T fcx = T(0), fcy = T(0), fcz = T(0);
      if (fast) {
        const T hz_ip = Hz[o + 1], hy_ip = Hy[o + 1];
        const T hz_jp = Hz[o + sx], hx_jp = Hx[o + sx];
        fcx = (hz_jp - hz) * (T)B.ih[1] - (hyn - hy) * (T)B.ih[2];
        fcy = (hxn - hx) * (T)B.ih[2] - (hz_ip - hz) * (T)B.ih[0];
        fcz = (hy_ip - hy) * (T)B.ih[0] - (hx_jp - hx) * (T)B.ih[1];
        cx = cy = cz = 0.0;
      } else {
        cx = cy = cz = 0.0;
        if (j <= ny && k <= nz)  // Ex (x-, y+, z+): dy Hz - dz Hy
          cx = dplus<T>(a, B, 1, Hz, o, sx, j, 1, i, j, k) - dplus<T>(a, B, 2, Hy, o, sxy, k, 1, i, j, k);
        if (i <= nx && k <= nz)  // Ey (x+, y-, z+): dz Hx - dx Hz
          cy = dplus<T>(a, B, 2, Hx, o, sxy, k, 0, i, j, k) - dplus<T>(a, B, 0, Hz, o, 1, i, 1, i, j, k);
        if (i <= nx && j <= ny)  // Ez (x+, y+, z-): dx Hy - dy Hx
          cz = dplus<T>(a, B, 0, Hy, o, 1, i, 0, i, j, k) - dplus<T>(a, B, 1, Hx, o, sx, j, 0, i, j, k);
        // absorbing faces: damping 2/(eta h) on tangential E nodes of the face
        if (B.abc_mask) {
          auto eta_at = [&](int comp) {
            double mu = B.mu_r0;
            if (B.mat & MAT_MU) {
              // node mean of mu over the cells containing the E node
              const int ck0 = clampi(k - 1, 0, nz - 1), ck1 = ck;
              double s = 0.0;
              if (comp == EX) s = (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj0, ck0) + (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj1, ck0) +
                                  (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj0, ck1) + (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj1, ck1);
              else if (comp == EY) s = (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj0, ck0) + (double)cell<T>(a.mat_mu, B.coff, B, ci1, cj0, ck0) +
                                       (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj0, ck1) + (double)cell<T>(a.mat_mu, B.coff, B, ci1, cj0, ck1);
              else s = (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj0, ck0) + (double)cell<T>(a.mat_mu, B.coff, B, ci1, cj0, ck0) +
                       (double)cell<T>(a.mat_mu, B.coff, B, ci0, cj1, ck0) + (double)cell<T>(a.mat_mu, B.coff, B, ci1, cj1, ck0);
              mu = 0.25 * s;
            }
            const double ep = comp == EX ? epx : (comp == EY ? epy : epz);
            return sqrt(a.mu0 * mu / ep);
          };
          const int r[3] = {i, j, k};
          for (int ax = 0; ax < 3; ++ax) {
            const bool lo = r[ax] == 0 && (B.abc_mask >> (2 * ax) & 1);
            const bool hi = r[ax] == B.n[ax] && (B.abc_mask >> (2 * ax + 1) & 1);
            const int m = (int)lo + (int)hi;
            if (!m) continue;
            const double g = m * 2.0 * B.ih[ax];
            if (ax != 0) sgx += g / eta_at(EX);
            if (ax != 1) sgy += g / eta_at(EY);
            if (ax != 2) sgz += g / eta_at(EZ);
          }
        }
      }
      // sources (current density inside the Cb bracket)
      double jx = 0.0, jy = 0.0, jz = 0.0;
      for (int q = 0; q < 2; ++q)
        if (sk[q] == k) {
          if (sc[q] == EX) jx += sv[q];
          else if (sc[q] == EY) jy += sv[q];
          else jz += sv[q];
        }
      // semi-implicit loss: Ca = (1-b)/(1+b), Cb = (dt/eps)/(1+b), b = dt sigma/(2 eps)
      const double bx = a.dt * sgx / (2.0 * epx), by = a.dt * sgy / (2.0 * epy), bz = a.dt * sgz / (2.0 * epz);
      const double cbx = (a.dt / epx) / (1.0 + bx), cby = (a.dt / epy) / (1.0 + by), cbz = (a.dt / epz) / (1.0 + bz);
      const double cax = (1.0 - bx) / (1.0 + bx), cay = (1.0 - by) / (1.0 + by), caz = (1.0 - bz) / (1.0 + bz);
      T nex = ex, ney = ey, nez = ez;
      if (fast) {
        nex = (T)cax * ex + (T)cbx * (fcx + (T)jx);
        ney = (T)cay * ey + (T)cby * (fcy + (T)jy);
        nez = (T)caz * ez + (T)cbz * (fcz + (T)jz);
      } else {
        if (j <= ny && k <= nz) nex = (T)(cax * (double)ex + cbx * (cx + jx));
        if (i <= nx && k <= nz) ney = (T)(cay * (double)ey + cby * (cy + jy));
        if (i <= nx && j <= ny) nez = (T)(caz * (double)ez + cbz * (cz + jz));
      }
      const double wzp = wplus(nz, k, B.h[2]), wzm = wminus(nz, k, B.h[2]);
      if (j <= ny && k <= nz) {
        Ex[o] = nex;
        eacc += 0.5 * epx * wxm * wyp * wzp * (double)nex * (double)nex;
      }
      if (i <= nx && k <= nz) {
        Ey[o] = ney;
        eacc += 0.5 * epy * wxp * wym * wzp * (double)ney * (double)ney;
      }
      if (i <= nx && j <= ny) {
        Ez[o] = nez;
        eacc += 0.5 * epz * wxp * wyp * wzm * (double)nez * (double)nez;
      }
      for (int q = 0; q < 2; ++q)
        if (pk[q] == k) {
          const T v = pc[q] == EX ? nex : (pc[q] == EY ? ney : nez);
          a.probes[(long long)pid[q] * a.pcap + nstep % a.pcap] = (double)v;
        }
      hx = hxn;
      hy = hyn;
      eA0 = eA1; eB0 = eB1; eC0 = eC1; eD0 = eD1;
      sA0 = sA1; sB0 = sB1; sC0 = sC1; sD0 = sD1;
    }
  }
  finish_energy(eacc, a, nstep, true);
}

// E part of W^n for the current fields (after a field write or a restore).
template <typename T>
__global__ __launch_bounds__(512) void k_e_energy(KArgs a) {
  double eacc = 0.0;
  const long long nstep = a.st->step;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile tl = a.tiles[t];
    const DevBlock& B = a.blocks[tl.block];
    const int i = tl.x0 + (int)threadIdx.x % a.tx;
    const int j = tl.y0 + (int)threadIdx.x / a.tx;
    const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
    if (i > nx + 1 || j > ny + 1) continue;
    const int k0 = tl.z0, k1 = min(tl.z0 + a.cz, nz + 2);
    const T* base = (const T*)a.pool + B.foff;
    const int ci0 = clampi(i - 1, 0, nx - 1), ci1 = clampi(i, 0, nx - 1);
    const int cj0 = clampi(j - 1, 0, ny - 1), cj1 = clampi(j, 0, ny - 1);
    const bool has_eps = B.mat & MAT_EPS;
    for (int k = k0; k < k1; ++k) {
      const long long o = i + B.sx * j + B.sxy * k;
      const int ck0 = clampi(k - 1, 0, nz - 1), ck1 = clampi(k, 0, nz - 1);
      auto ev = [&](int ci, int cj, int ck) {
        return has_eps ? (double)cell<T>(a.mat_eps, B.coff, B, ci, cj, ck) : B.eps_r0;
      };
      const double epx = a.eps0 * (0.25 * ((ev(ci0, cj0, ck0) + ev(ci0, cj1, ck0)) + (ev(ci0, cj0, ck1) + ev(ci0, cj1, ck1))));
      const double epy = a.eps0 * (0.25 * ((ev(ci0, cj0, ck0) + ev(ci1, cj0, ck0)) + (ev(ci0, cj0, ck1) + ev(ci1, cj0, ck1))));
      const double epz = a.eps0 * (0.25 * ((ev(ci0, cj0, ck0) + ev(ci1, cj0, ck0)) + (ev(ci0, cj1, ck0) + ev(ci1, cj1, ck0))));
      const double wxp = wplus(nx, i, B.h[0]), wxm = wminus(nx, i, B.h[0]);
      const double wyp = wplus(ny, j, B.h[1]), wym = wminus(ny, j, B.h[1]);
      const double wzp = wplus(nz, k, B.h[2]), wzm = wminus(nz, k, B.h[2]);
      if (j <= ny && k <= nz) { const double v = (double)base[o]; eacc += 0.5 * epx * wxm * wyp * wzp * v * v; }
      if (i <= nx && k <= nz) { const double v = (double)base[B.csz + o]; eacc += 0.5 * epy * wxp * wym * wzp * v * v; }
      if (i <= nx && j <= ny) { const double v = (double)base[2 * B.csz + o]; eacc += 0.5 * epz * wxp * wyp * wzm * v * v; }
    }
  }
  // write slot n (not n+1): shift the step seen by finish_energy by one
  finish_energy(eacc, a, nstep - 1, true);
}

// ------------------------------------------------------- interface gather
// Fills the face buffers: for every own face node, the neighbour's
// tangential field on its coincident face, through the per-axis taps
// (identity at 1:1; the norm-compatible 1:2 interpolation otherwise).
// Accumulated in fp64.
template <typename T>
__global__ __launch_bounds__(256) void k_face_gather(const DevBlock* blocks, const FaceJob* jobs,
                                                     const Taps* taps, const void* pool,
                                                     double* face) {
  const FaceJob J = jobs[blockIdx.y];
  const DevBlock& B = blocks[J.block];
  const DevBlock& N = blocks[J.nb];
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)J.ext[0] * J.ext[1];
  if (id >= tot) return;
  const int r0 = (int)(id % J.ext[0]), r1 = (int)(id / J.ext[0]);
  const Taps& T0 = taps[J.taps_off[0] + r0];
  const Taps& T1 = taps[J.taps_off[1] + r1];
  const T* nf = (const T*)pool + N.foff + (long long)J.comp * N.csz;
  const long long st[3] = {1, N.sx, N.sxy};
  const int axis = J.face >> 1;
  const long long onrm = (long long)J.nb_idx * st[axis];
  double v = 0.0;
  for (int q = 0; q < T1.count; ++q) {
    double s = 0.0;
    const long long o1 = onrm + (long long)(T1.start + q) * st[J.t_axis[1]];
    for (int p = 0; p < T0.count; ++p)
      s += T0.w[p] * (double)nf[o1 + (long long)(T0.start + p) * st[J.t_axis[0]]];
    v += T1.w[q] * s;
  }
  // own face-node index in the node-box face layout
  const int bx = B.n[0] + 2, by = B.n[1] + 2;
  long long fidx;
  if (axis == 0) fidx = (long long)r0 + (long long)by * r1;       // (j, k)
  else fidx = (long long)r0 + (long long)bx * r1;                 // (i, k) or (i, j)
  face[B.fboff[J.face] + (long long)(J.is_h * 2 + J.slot) * B.fsz[J.face] + fidx] = v;
}

// ------------------------------------------------------------- launchers
template <typename T>
hipError_t launch_h(const KArgs& a, int grid, int threads, hipStream_t s) {
  hipLaunchKernelGGL(k_h_update<T>, dim3(grid), dim3(threads), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_e(const KArgs& a, int grid, int threads, hipStream_t s) {
  hipLaunchKernelGGL(k_e_update<T>, dim3(grid), dim3(threads), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_e_energy(const KArgs& a, int grid, int threads, hipStream_t s) {
  hipLaunchKernelGGL(k_e_energy<T>, dim3(grid), dim3(threads), 0, s, a);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_gather(const DevBlock* blocks, const FaceJob* jobs, int njobs, int max_nodes,
                         const Taps* taps, const void* pool, double* face, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  dim3 grid((max_nodes + 255) / 256, njobs);
  hipLaunchKernelGGL(k_face_gather<T>, grid, dim3(256), 0, s, blocks, jobs, taps, pool, face);
  return hipGetLastError();
}

template hipError_t launch_h<float>(const KArgs&, int, int, hipStream_t);
template hipError_t launch_h<double>(const KArgs&, int, int, hipStream_t);
template hipError_t launch_e<float>(const KArgs&, int, int, hipStream_t);
template hipError_t launch_e<double>(const KArgs&, int, int, hipStream_t);
template hipError_t launch_e_energy<float>(const KArgs&, int, int, hipStream_t);
template hipError_t launch_e_energy<double>(const KArgs&, int, int, hipStream_t);
template hipError_t launch_gather<float>(const DevBlock*, const FaceJob*, int, int, const Taps*, const void*, double*, hipStream_t);
template hipError_t launch_gather<double>(const DevBlock*, const FaceJob*, int, int, const Taps*, const void*, double*, hipStream_t);

}  // namespace sbp
