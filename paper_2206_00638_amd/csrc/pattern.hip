// Access-pattern probes of the two update kernels (a measurement reference,
// like a device-to-device copy; not part of the stepping library).
//
// On one block's node box, in the library's layout (x fastest, rows of
// n + 2 nodes, planes padded to a multiple of 64 nodes, six component arrays
// of a pool, and the per-cell permittivity of a block with few distinct
// values: a byte per cell indexing a table staged in LDS), each probe issues the
// loads and stores per node of the H update or of the E update of a plain
// block with per-cell permittivity: the same tiles (`threads` consecutive
// nodes of a plane over `cz` planes, one thread per node column marching up
// through the planes with the next plane's loads issued first), the same
// grouped walk of the tile list over the XCDs and 32-bit offsets from the
// component base.  It computes the interior two-point differences on every
// node and writes the updated field, with no closure rows, energy sums,
// probes or sources.  The time per launch therefore bounds what the update
// kernels can reach with their access pattern on this part.
//
// A third probe keeps the E update's streams and drops its neighbours: per
// node it reads the six field components and the cell's permittivity and
// writes the three E components back in place, on the same tiles and walk.
// It bounds any kernel that moves those bytes in that mix of reads and
// in-place writes, stencil or not.  Every cell indexes table entry 0 (1.0).
//
// sbp_pattern_time(n, threads, cz, reps, out_ms): an n^3-cell block in fp32,
// buffers allocated and freed here; out_ms[0], out_ms[1], out_ms[2] = mean
// time per launch of the H, E and stream probes over `reps` launches (after
// two warm-up launches each), by HIP events on a stream of its own.  Returns
// 0, or the HIP error code of the first failing call.
#include <hip/hip_runtime.h>

namespace {

constexpr int kXcds = 8;   // workgroups are dispatched round-robin over the XCDs
constexpr int kGroup = 8;  // consecutive tiles per XCD group
constexpr int kTab = 64;   // permittivity table entries

struct Walk {
  int t, stride;
  __device__ Walk(int ntiles) {
    const int g = blockIdx.x, G = gridDim.x;
    const int w = g / kXcds, x = g % kXcds, full = (G / kXcds) / kGroup * kGroup;
    t = w < full ? ((w / kGroup) * kXcds + x) * kGroup + w % kGroup : g;
    stride = G;
    (void)ntiles;
  }
};

struct Box {
  int n, sx, ny2, nz2;
  unsigned sxy, csz;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// H pattern: E and H at the node, E one node back along y and x, E one plane
// back (carried); H written.
__global__ __launch_bounds__(256) void k_pattern_h(float* pool, Box b, int threads, int cz, int ntiles, float c) {
  const float* Ex = pool;
  const float* Ey = pool + b.csz;
  const float* Ez = pool + 2ull * b.csz;
  float* Hx = pool + 3ull * b.csz;
  float* Hy = pool + 4ull * b.csz;
  float* Hz = pool + 5ull * b.csz;
  const int tpp = (b.sx * b.ny2 + threads - 1) / threads;
  for (Walk it(ntiles); it.t < ntiles; it.t += it.stride) {
    const int slab = it.t / tpp, tq = it.t - slab * tpp;
    const int q = tq * threads + (int)threadIdx.x;
    if ((int)threadIdx.x >= threads || q >= b.sx * b.ny2) continue;
    const int j = q / b.sx, i = q - j * b.sx;
    const int k0 = slab * cz, k1 = min(k0 + cz, b.nz2);
    unsigned u = (unsigned)q + b.sxy * (unsigned)k0;
    const unsigned dy = j > 0 ? (unsigned)b.sx : 0u, dx = i > 0 ? 1u : 0u;
    float exz = k0 > 0 ? Ex[u - b.sxy] : Ex[u], eyz = k0 > 0 ? Ey[u - b.sxy] : Ey[u];
    float ex = Ex[u], ey = Ey[u], ez = Ez[u], hx = Hx[u], hy = Hy[u], hz = Hz[u];
    float ezy = Ez[u - dy], exy = Ex[u - dy], ezx = Ez[u - dx], eyx = Ey[u - dx];
    for (int k = k0; k < k1; ++k, u += b.sxy) {
      float nex = 0.f, ney = 0.f, nez = 0.f, nhx = 0.f, nhy = 0.f, nhz = 0.f, nezy = 0.f, nexy = 0.f, nezx = 0.f,
            neyx = 0.f;
      if (k + 1 < k1) {
        const unsigned v = u + b.sxy;
        nex = Ex[v];
        ney = Ey[v];
        nez = Ez[v];
        nhx = Hx[v];
        nhy = Hy[v];
        nhz = Hz[v];
        nezy = Ez[v - dy];
        nexy = Ex[v - dy];
        nezx = Ez[v - dx];
        neyx = Ey[v - dx];
      }
      Hx[u] = hx + c * ((ey - eyz) - (ez - ezy));
      Hy[u] = hy + c * ((ez - ezx) - (ex - exz));
      Hz[u] = hz + c * ((ex - exy) - (ey - eyx));
      exz = ex;
      eyz = ey;
      ex = nex;
      ey = ney;
      ez = nez;
      hx = nhx;
      hy = nhy;
      hz = nhz;
      ezy = nezy;
      exy = nexy;
      ezx = nezx;
      eyx = neyx;
    }
  }
}

// E pattern: E and H at the node, H one node ahead along y and x, H one plane
// ahead (the next plane's centre values, carried), the four permittivity
// cells of each plane (the previous plane's carried); E written.
__global__ __launch_bounds__(256) void k_pattern_e(float* pool, const unsigned char* cells, const float* tab, Box b,
                                                  int threads, int cz, int ntiles, float c) {
  __shared__ float etab[kTab];
  if (threadIdx.x < kTab) etab[threadIdx.x] = tab[threadIdx.x];
  __syncthreads();
  float* Ex = pool;
  float* Ey = pool + b.csz;
  float* Ez = pool + 2ull * b.csz;
  const float* Hx = pool + 3ull * b.csz;
  const float* Hy = pool + 4ull * b.csz;
  const float* Hz = pool + 5ull * b.csz;
  const int n = b.n, cp = n * n;
  const int tpp = (b.sx * b.ny2 + threads - 1) / threads;
  for (Walk it(ntiles); it.t < ntiles; it.t += it.stride) {
    const int slab = it.t / tpp, tq = it.t - slab * tpp;
    const int q = tq * threads + (int)threadIdx.x;
    if ((int)threadIdx.x >= threads || q >= b.sx * b.ny2) continue;
    const int j = q / b.sx, i = q - j * b.sx;
    const int k0 = slab * cz, k1 = min(k0 + cz, b.nz2);
    const int ci0 = clampi(i - 1, 0, n - 1), ci1 = clampi(i, 0, n - 1);
    const int cj0 = clampi(j - 1, 0, n - 1), cj1 = clampi(j, 0, n - 1);
    const int A = ci0 + n * cj0, cdx = ci1 - ci0, cdy = (cj1 - cj0) * n;
    const unsigned dy = j <= n ? (unsigned)b.sx : 0u, dx = i <= n ? 1u : 0u;
    unsigned u = (unsigned)q + b.sxy * (unsigned)k0;
    const unsigned char* p0 = cells + A + cp * clampi(k0 - 1, 0, n - 1);
    float e0a = etab[p0[0]], e0b = etab[p0[cdx]], e0c = etab[p0[cdy]], e0d = etab[p0[cdx + cdy]];
    float hx = Hx[u], hy = Hy[u];
    // the cells' table indices stay in registers until their plane is updated
    auto load = [&](unsigned v, int k, float& ex, float& ey, float& ez, float& hz, float& hyz, float& hxz, float& hzy,
                    float& hxy, float& hzx, float& hyx, unsigned& e1a, unsigned& e1b, unsigned& e1c, unsigned& e1d) {
      const unsigned vz = v + (k <= n ? b.sxy : 0u);
      ex = Ex[v];
      ey = Ey[v];
      ez = Ez[v];
      hz = Hz[v];
      hyz = Hy[vz];
      hxz = Hx[vz];
      hzy = Hz[v + dy];
      hxy = Hx[v + dy];
      hzx = Hz[v + dx];
      hyx = Hy[v + dx];
      const unsigned char* p1 = cells + A + cp * clampi(k, 0, n - 1);
      e1a = p1[0];
      e1b = p1[cdx];
      e1c = p1[cdy];
      e1d = p1[cdx + cdy];
    };
    float ex, ey, ez, hz, hyz, hxz, hzy, hxy, hzx, hyx;
    unsigned i1a, i1b, i1c, i1d;
    load(u, k0, ex, ey, ez, hz, hyz, hxz, hzy, hxy, hzx, hyx, i1a, i1b, i1c, i1d);
    for (int k = k0; k < k1; ++k, u += b.sxy) {
      float nex = 0.f, ney = 0.f, nez = 0.f, nhz = 0.f, nhyz = 0.f, nhxz = 0.f, nhzy = 0.f, nhxy = 0.f, nhzx = 0.f,
            nhyx = 0.f;
      unsigned n1a = 0, n1b = 0, n1c = 0, n1d = 0;
      if (k + 1 < k1) load(u + b.sxy, k + 1, nex, ney, nez, nhz, nhyz, nhxz, nhzy, nhxy, nhzx, nhyx, n1a, n1b, n1c, n1d);
      const float e1a = etab[i1a], e1b = etab[i1b], e1c = etab[i1c], e1d = etab[i1d];
      const float mx = (e0a + e0c) + (e1a + e1c), my = (e0a + e0b) + (e1a + e1b), mz = (e0a + e0b) + (e0c + e0d);
      Ex[u] = ex + c / mx * ((hzy - hz) - (hyz - hy));
      Ey[u] = ey + c / my * ((hxz - hx) - (hzx - hz));
      Ez[u] = ez + c / mz * ((hyx - hy) - (hxy - hx));
      hx = hxz;
      hy = hyz;
      e0a = e1a;
      e0b = e1b;
      e0c = e1c;
      e0d = e1d;
      ex = nex;
      ey = ney;
      ez = nez;
      hz = nhz;
      hyz = nhyz;
      hxz = nhxz;
      hzy = nhzy;
      hxy = nhxy;
      hzx = nhzx;
      hyx = nhyx;
      i1a = n1a;
      i1b = n1b;
      i1c = n1c;
      i1d = n1d;
    }
  }
}

// Stream probe: the E update's reads and in-place writes at the node only.
__global__ __launch_bounds__(256) void k_pattern_streams(float* pool, const unsigned char* cells, const float* tab,
                                                        Box b, int threads, int cz, int ntiles, float c) {
  __shared__ float etab[kTab];
  if (threadIdx.x < kTab) etab[threadIdx.x] = tab[threadIdx.x];
  __syncthreads();
  float* Ex = pool;
  float* Ey = pool + b.csz;
  float* Ez = pool + 2ull * b.csz;
  const float* Hx = pool + 3ull * b.csz;
  const float* Hy = pool + 4ull * b.csz;
  const float* Hz = pool + 5ull * b.csz;
  const int n = b.n, cp = n * n;
  const int tpp = (b.sx * b.ny2 + threads - 1) / threads;
  for (Walk it(ntiles); it.t < ntiles; it.t += it.stride) {
    const int slab = it.t / tpp, tq = it.t - slab * tpp;
    const int q = tq * threads + (int)threadIdx.x;
    if ((int)threadIdx.x >= threads || q >= b.sx * b.ny2) continue;
    const int j = q / b.sx, i = q - j * b.sx;
    const int k0 = slab * cz, k1 = min(k0 + cz, b.nz2);
    const int A = clampi(i, 0, n - 1) + n * clampi(j, 0, n - 1);
    unsigned u = (unsigned)q + b.sxy * (unsigned)k0;
    for (int k = k0; k < k1; ++k, u += b.sxy) {
      const float e = c / etab[cells[A + cp * clampi(k, 0, n - 1)]];
      const float hx = Hx[u], hy = Hy[u], hz = Hz[u];
      Ex[u] = Ex[u] + e * (hy - hz);
      Ey[u] = Ey[u] + e * (hz - hx);
      Ez[u] = Ez[u] + e * (hx - hy);
    }
  }
}

}  // namespace

extern "C" int sbp_pattern_time(int n, int threads, int cz, int reps, double out_ms[3]) {
  if (n < 4 || n > 1024 || (threads != 64 && threads != 128 && threads != 256) || cz < 1 || reps < 1 || !out_ms)
    return (int)hipErrorInvalidValue;
  Box b;
  b.n = n;
  b.sx = n + 2;
  b.ny2 = n + 2;
  b.nz2 = n + 2;
  b.sxy = (unsigned)(((long long)b.sx * b.ny2 + 63) / 64 * 64);
  b.csz = b.sxy * (unsigned)b.nz2;
  const size_t pool_bytes = 6ull * b.csz * sizeof(float), cell_bytes = (size_t)n * n * n;
  const int tpp = (b.sx * b.ny2 + threads - 1) / threads, slabs = (b.nz2 + cz - 1) / cz;
  const int ntiles = tpp * slabs, grid = (ntiles + 7) / 8 * 8;
  float *pool = nullptr, *tab = nullptr;
  unsigned char* cells = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipSuccess;
  auto run = [&]() -> hipError_t {
    hipError_t e;
    if ((e = hipMalloc(&pool, pool_bytes)) != hipSuccess) return e;
    if ((e = hipMalloc(&cells, cell_bytes)) != hipSuccess) return e;
    if ((e = hipMalloc(&tab, kTab * sizeof(float))) != hipSuccess) return e;
    if ((e = hipStreamCreate(&s)) != hipSuccess) return e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(pool, 0, pool_bytes, s)) != hipSuccess) return e;
    // every cell indexes entry 0, unit permittivity (0x3f800000 = 1.0f): a
    // finite quotient per node
    if ((e = hipMemsetAsync(cells, 0, cell_bytes, s)) != hipSuccess) return e;
    if ((e = hipMemsetD32Async((hipDeviceptr_t)tab, 0x3f800000, kTab, s)) != hipSuccess) return e;
    for (int which = 0; which < 3; ++which) {
      auto launch = [&]() {
        if (which == 0)
          hipLaunchKernelGGL(k_pattern_h, dim3(grid), dim3(threads), 0, s, pool, b, threads, cz, ntiles, 1e-3f);
        else if (which == 1)
          hipLaunchKernelGGL(k_pattern_e, dim3(grid), dim3(threads), 0, s, pool, cells, tab, b, threads, cz, ntiles,
                             1e-3f);
        else
          hipLaunchKernelGGL(k_pattern_streams, dim3(grid), dim3(threads), 0, s, pool, cells, tab, b, threads, cz,
                             ntiles, 1e-3f);
      };
      launch();
      launch();
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
      for (int r = 0; r < reps; ++r) launch();
      if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
      out_ms[which] = ms / reps;
    }
    return hipSuccess;
  };
  err = run();
  if (s) (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (cells) (void)hipFree(cells);
  if (tab) (void)hipFree(tab);
  if (pool) (void)hipFree(pool);
  return (int)err;
}
