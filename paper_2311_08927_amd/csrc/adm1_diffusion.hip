// Diffusion between the AD particles with a uniform-grid neighbour search.
//
// The paper couples the particles only through advection (sec. 2.3) and names
// diffusion as the next step without fixing an operator.  This file takes the
// standard SPH diffusion operator on equal particle volumes V_p (sec. 2.3:
// tank volume over particle count):
//     dC_i/dt = 2 D V_p sum_{j != i, r_ij < 2h} (C_i - C_j) W'(r_ij) / r_ij,
// with the 3-D Wendland C2 kernel, W'(r)/r = -5 a / h^2 (1 - r/(2h))^3,
// a = 21 / (16 pi h^3), on the 13 soluble differential entries, advanced by
// explicit Euler substeps.
//
// Neighbour search: cells of edge h (half the kernel support) over a fixed
// box, so every neighbour of a particle lies in the 5 x 5 x 5 cells around
// its own (a search volume of 125 h^3 against 216 h^3 with cells of edge
// 2h).  Per
// call (positions are fixed over the interval):
//   k_grid_count   -- cell of every particle (clamped into the box), counts;
//   k_scan_*       -- exclusive prefix sums of the counts (cell starts);
//   k_grid_place   -- scatter of the particle indices into cell order;
//   k_grid_sort    -- one thread per cell sorts its indices ascending, so the
//                     order, and with it every sum, is the same run to run;
//   k_gather_pos   -- positions in cell order, one float4 per particle, and
//                     the inverse permutation (each particle's slot);
//   k_gather_c     -- the soluble entries into cell order, one 128-byte row
//                     of kCRow doubles per particle (state read coalesced in
//                     particle order, rows written to the particles' slots);
// then per substep k_diffuse, one thread per particle in cell order
// (neighbouring threads read the same cells), sums over those cells (25
// index ranges: the five cells of a row along x are consecutive) and writes
// the Euler-updated row into a second buffer; the two buffers swap between
// substeps, and k_scatter_c writes the last rows back to the state in
// particle order (coalesced).  A
// candidate is first tested in FP32 against a slightly enlarged radius; the
// FP64 test then decides, so the neighbour sets are those of an FP64
// distance test.  Every launch is bounded by n or by the cell count; indices
// read back from the grid are < n by construction.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <new>
#include <utility>

#include "adm1.h"

namespace adm1 {
namespace {

constexpr int kDiffRows = 13;
// cells of edge 2h / kSub: the support 2h spans kSub cells each way
constexpr int kSub = 2;
constexpr int kCRow = 16;  // doubles per particle row of the cell-ordered copy
constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanChunk = kScanThreads * kScanPer;

// state rows of the soluble differential entries
__device__ __forceinline__ int diff_row(int k)
{
    constexpr int rows[kDiffRows] = {0, 1, 2, 3, 4, 5, 6, 8, 9, 10, 11, 24, 25};
    return rows[k];
}

struct GridGeom {
    double lo[3];
    double inv_cs[3];
    int nc[3];
};

__device__ __forceinline__ int axis_cell(double x, double lo, double inv_cs, int nc)
{
    double v = floor((x - lo) * inv_cs);
    if (!(v >= 0.0)) v = 0.0;  // below the box, or NaN
    if (v > (double)(nc - 1)) v = (double)(nc - 1);
    return (int)v;
}

__device__ __forceinline__ void cell_coords(const GridGeom& g, float x, float y, float z, int& cx,
                                            int& cy, int& cz)
{
    cx = axis_cell((double)x, g.lo[0], g.inv_cs[0], g.nc[0]);
    cy = axis_cell((double)y, g.lo[1], g.inv_cs[1], g.nc[1]);
    cz = axis_cell((double)z, g.lo[2], g.inv_cs[2], g.nc[2]);
}

__global__ void __launch_bounds__(256) k_grid_count(const float* __restrict__ pos, int64_t ld,
                                                    int64_t n, GridGeom g,
                                                    int32_t* __restrict__ cell,
                                                    int32_t* __restrict__ count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cx, cy, cz;
    cell_coords(g, pos[i], pos[ld + i], pos[2 * ld + i], cx, cy, cz);
    const int c = (cz * g.nc[1] + cy) * g.nc[0] + cx;
    cell[i] = c;
    atomicAdd(&count[c], 1);
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Exclusive scan, level 1: each block scans kScanChunk counts into `start`
// and writes its total to bsum[block].
__global__ void __launch_bounds__(kScanThreads) k_scan_local(const int32_t* __restrict__ count,
                                                             int64_t m,
                                                             int32_t* __restrict__ start,
                                                             int32_t* __restrict__ bsum)
{
    __shared__ int32_t s[2][kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer], tot = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < m ? count[base + k] : 0;
        tot += v[k];
    }
    int cur = 0;
    s[0][threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int32_t x = s[cur][threadIdx.x] +
                          ((int)threadIdx.x >= off ? s[cur][threadIdx.x - off] : 0);
        s[cur ^ 1][threadIdx.x] = x;
        cur ^= 1;
        __syncthreads();
    }
    int32_t run = s[cur][threadIdx.x] - tot;  // exclusive prefix of this thread
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < m) start[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanThreads - 1) bsum[blockIdx.x] = s[cur][threadIdx.x];
}

// Level 2: one block scans the block totals in place (exclusive), in chunks
// of its width with a running carry, and writes the grand total to
// start[m].
__global__ void __launch_bounds__(kScanThreads) k_scan_top(int32_t* __restrict__ bsum,
                                                           int64_t nb,
                                                           int32_t* __restrict__ start,
                                                           int64_t m)
{
    __shared__ int32_t s[2][kScanThreads];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
        const int64_t j = c0 + threadIdx.x;
        const int32_t v = j < nb ? bsum[j] : 0;
        int cur = 0;
        s[0][threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kScanThreads; off <<= 1) {
            const int32_t x = s[cur][threadIdx.x] +
                              ((int)threadIdx.x >= off ? s[cur][threadIdx.x - off] : 0);
            s[cur ^ 1][threadIdx.x] = x;
            cur ^= 1;
            __syncthreads();
        }
        const int32_t c = carry;
        if (j < nb) bsum[j] = c + s[cur][threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kScanThreads - 1) carry = c + s[cur][threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) start[m] = carry;
}

__global__ void __launch_bounds__(256) k_scan_add(int32_t* __restrict__ start, int64_t m,
                                                  const int32_t* __restrict__ bsum)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) start[i] += bsum[i / kScanChunk];
}

__global__ void __launch_bounds__(256) k_grid_place(const int32_t* __restrict__ cell, int64_t n,
                                                    const int32_t* __restrict__ start,
                                                    int32_t* __restrict__ cursor,
                                                    int32_t* __restrict__ sorted)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell[i];
    sorted[start[c] + atomicAdd(&cursor[c], 1)] = (int32_t)i;
}

// Insertion sort of each cell's indices (cells hold a few tens of particles).
__global__ void __launch_bounds__(256) k_grid_sort(const int32_t* __restrict__ start,
                                                   int64_t m, int32_t* __restrict__ sorted)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    const int32_t b = start[c], e = start[c + 1];
    for (int32_t a = b + 1; a < e; ++a) {
        const int32_t v = sorted[a];
        int32_t k = a - 1;
        while (k >= b && sorted[k] > v) {
            sorted[k + 1] = sorted[k];
            --k;
        }
        sorted[k + 1] = v;
    }
}

__global__ void __launch_bounds__(256) k_gather_pos(const int32_t* __restrict__ sorted,
                                                    const float* __restrict__ pos, int64_t ld,
                                                    int64_t n, float4* __restrict__ spos,
                                                    int32_t* __restrict__ slot)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = sorted[s];
    spos[s] = float4{pos[i], pos[ld + i], pos[2 * ld + i], 0.0f};
    slot[i] = (int32_t)s;
}

// Particle order: coalesced reads of the state, one row write per particle.
__global__ void __launch_bounds__(256) k_gather_c(const int32_t* __restrict__ slot,
                                                  const double* __restrict__ state, int64_t ld,
                                                  int64_t n, double* __restrict__ sc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double* row = sc + (int64_t)slot[i] * kCRow;
#pragma unroll
    for (int k = 0; k < kDiffRows; ++k) row[k] = state[diff_row(k) * ld + i];
}

// Particle order: one row read per particle, coalesced writes of the state.
__global__ void __launch_bounds__(256) k_scatter_c(const int32_t* __restrict__ slot,
                                                   const double* __restrict__ sc, int64_t n,
                                                   double* __restrict__ state, int64_t ld)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* row = sc + (int64_t)slot[i] * kCRow;
#pragma unroll
    for (int k = 0; k < kDiffRows; ++k) state[diff_row(k) * ld + i] = row[k];
}

struct DiffArgs {
    GridGeom g;
    const int32_t* start;
    const int32_t* sorted;
    const float4* spos;
    const double* sc;  // [n_max][kCRow] rows in cell order, read
    double* out;       // [n_max][kCRow] updated rows, written
    int64_t n;
    float h2x4_pre;  // (2h)^2 (1 + 1e-4): FP32 prefilter, never below the FP64 test
    double h2x4;     // (2h)^2
    double inv_h;
    double fcoef;    // -5 a / h^2
    double scale;    // substep x 2 D V_p
    int32_t* neighbours;
};

__global__ void __launch_bounds__(256) k_diffuse(DiffArgs a)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n) return;
    const float4 ps = a.spos[s];
    const float xs = ps.x, ys = ps.y, zs = ps.z;
    double cs[kDiffRows], acc[kDiffRows];
#pragma unroll
    for (int k = 0; k < kDiffRows; ++k) {
        cs[k] = a.sc[s * kCRow + k];
        acc[k] = 0.0;
    }
    int cx, cy, cz;
    cell_coords(a.g, xs, ys, zs, cx, cy, cz);
    int cnt = 0;
    for (int dz = -kSub; dz <= kSub; ++dz) {
        const int z = cz + dz;
        if (z < 0 || z >= a.g.nc[2]) continue;
        for (int dy = -kSub; dy <= kSub; ++dy) {
            const int y = cy + dy;
            if (y < 0 || y >= a.g.nc[1]) continue;
            // the cells x-kSub..x+kSub of a row are consecutive in cell
            // order, and so are their particles: one index range per row
            const int x0 = cx > kSub ? cx - kSub : 0;
            const int x1 = cx + kSub < a.g.nc[0] ? cx + kSub : a.g.nc[0] - 1;
            const int c0 = (z * a.g.nc[1] + y) * a.g.nc[0] + x0;
            const int32_t e = a.start[c0 + (x1 - x0) + 1];
            for (int32_t j = a.start[c0]; j < e; ++j) {
                if (j == s) continue;
                const float4 pj = a.spos[j];
                const float fx = xs - pj.x, fy = ys - pj.y, fz = zs - pj.z;
                if (!(fx * fx + fy * fy + fz * fz < a.h2x4_pre)) continue;
                const double ddx = (double)xs - (double)pj.x;
                const double ddy = (double)ys - (double)pj.y;
                const double ddz = (double)zs - (double)pj.z;
                const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                if (!(r2 < a.h2x4)) continue;
                const double t = 1.0 - 0.5 * sqrt(r2) * a.inv_h;
                const double F = a.fcoef * t * t * t;
                ++cnt;
                const double* cj = a.sc + (int64_t)j * kCRow;
#pragma unroll
                for (int k = 0; k < kDiffRows; ++k) acc[k] = fma(cs[k] - cj[k], F, acc[k]);
            }
        }
    }
    double* row = a.out + s * kCRow;
#pragma unroll
    for (int k = 0; k < kDiffRows; ++k) row[k] = fma(a.scale, acc[k], cs[k]);
    if (a.neighbours) a.neighbours[a.sorted[s]] = cnt;
}

bool is_dev(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
           at.type == hipMemoryTypeUnified;
}

inline unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace
}  // namespace adm1

struct adm1_grid {
    adm1_diffusion d;
    adm1::GridGeom g;
    int64_t n_max, ncell, nblk;
    int32_t *cell, *count, *start, *sorted, *bsum, *slot;
    float4* spos;
    double *sc, *sc2;
};

extern "C" {

int adm1_grid_create(const adm1_diffusion* d, int64_t n_max, adm1_grid** out)
{
    if (!d || !out) return ADM1_E_NULL;
    *out = nullptr;
    if (n_max < 1 || n_max > INT32_MAX) return ADM1_E_SIZE;
    if (!(d->h > 0.0) || !std::isfinite(d->h) || !(d->D >= 0.0) || !std::isfinite(d->D) ||
        !(d->V_p > 0.0) || !std::isfinite(d->V_p))
        return ADM1_E_OPTS;
    adm1::GridGeom g;
    double cells = 1.0;
    for (int k = 0; k < 3; ++k) {
        const double ext = d->hi[k] - d->lo[k];
        if (!(ext > 0.0) || !std::isfinite(ext) || !std::isfinite(d->lo[k])) return ADM1_E_OPTS;
        const double cs = 2.0 * d->h / adm1::kSub;
        const double nc = std::ceil(ext / cs);
        if (nc > (double)(1 << 20)) return ADM1_E_OPTS;
        g.nc[k] = nc < 1.0 ? 1 : (int)nc;
        g.lo[k] = d->lo[k];
        g.inv_cs[k] = 1.0 / cs;
        cells *= g.nc[k];
    }
    if (cells > (double)(1 << 26)) return ADM1_E_OPTS;
    adm1_grid* p = new (std::nothrow) adm1_grid;
    if (!p) return ADM1_E_NOMEM;
    p->d = *d;
    p->g = g;
    p->n_max = n_max;
    p->ncell = (int64_t)cells;
    p->nblk = (p->ncell + adm1::kScanChunk - 1) / adm1::kScanChunk;
    p->cell = p->count = p->start = p->sorted = p->bsum = p->slot = nullptr;
    p->spos = nullptr;
    p->sc = p->sc2 = nullptr;
    bool ok = hipMalloc((void**)&p->cell, n_max * sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void**)&p->sorted, n_max * sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void**)&p->count, p->ncell * sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void**)&p->start, (p->ncell + 1) * sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void**)&p->bsum, p->nblk * sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void**)&p->spos, n_max * sizeof(float4)) == hipSuccess &&
              hipMalloc((void**)&p->slot, n_max * sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void**)&p->sc, adm1::kCRow * n_max * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&p->sc2, adm1::kCRow * n_max * sizeof(double)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        adm1_grid_destroy(p);
        return ADM1_E_NOMEM;
    }
    *out = p;
    return ADM1_OK;
}

void adm1_grid_destroy(adm1_grid* g)
{
    if (!g) return;
    for (void* q : {(void*)g->cell, (void*)g->count, (void*)g->start, (void*)g->sorted,
                    (void*)g->bsum, (void*)g->slot, (void*)g->spos, (void*)g->sc,
                    (void*)g->sc2})
        if (q) (void)hipFree(q);
    delete g;
}

int adm1_diffuse(adm1_grid* g, double* state, int64_t ld, const float* pos, int64_t n,
                 double dt_days, int32_t substeps, int32_t* neighbours, void* stream)
{
    using namespace adm1;
    if (!g || !state || !pos) return ADM1_E_NULL;
    if (n < 0 || n > g->n_max || ld < n || ld <= 0 || ld % 64 != 0) return ADM1_E_SIZE;
    if (!(dt_days > 0.0) || !std::isfinite(dt_days)) return ADM1_E_DT;
    if (substeps < 1 || substeps > (1 << 20)) return ADM1_E_OPTS;
    if (!is_dev(state) || !is_dev(pos) || (neighbours && !is_dev(neighbours)))
        return ADM1_E_NOT_DEVICE;
    if (n == 0) return ADM1_OK;
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = g->ncell;
    // cell of every particle and cell counts
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(m, 256)), dim3(256), 0, s, g->count, m, 0);
    hipLaunchKernelGGL(k_grid_count, dim3(blocks(n, 256)), dim3(256), 0, s, pos, ld, n, g->g,
                       g->cell, g->count);
    // cell starts
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)g->nblk), dim3(kScanThreads), 0, s,
                       g->count, m, g->start, g->bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, g->bsum, g->nblk,
                       g->start, m);
    hipLaunchKernelGGL(k_scan_add, dim3(blocks(m, 256)), dim3(256), 0, s, g->start, m, g->bsum);
    // indices in cell order, ascending within a cell
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(m, 256)), dim3(256), 0, s, g->count, m, 0);
    hipLaunchKernelGGL(k_grid_place, dim3(blocks(n, 256)), dim3(256), 0, s, g->cell, n,
                       g->start, g->count, g->sorted);
    hipLaunchKernelGGL(k_grid_sort, dim3(blocks(m, 256)), dim3(256), 0, s, g->start, m,
                       g->sorted);
    hipLaunchKernelGGL(k_gather_pos, dim3(blocks(n, 256)), dim3(256), 0, s, g->sorted, pos, ld,
                       n, g->spos, g->slot);
    hipLaunchKernelGGL(k_gather_c, dim3(blocks(n, 256)), dim3(256), 0, s, g->slot, state, ld, n,
                       g->sc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    const double h = g->d.h;
    DiffArgs a;
    a.g = g->g;
    a.start = g->start;
    a.sorted = g->sorted;
    a.spos = g->spos;
    a.n = n;
    a.h2x4 = 4.0 * h * h;
    a.h2x4_pre = (float)(a.h2x4 * (1.0 + 1e-4));
    a.inv_h = 1.0 / h;
    a.fcoef = -5.0 * (21.0 / (16.0 * M_PI * h * h * h)) / (h * h);
    a.scale = dt_days / substeps * 2.0 * g->d.D * g->d.V_p;
    double* cur = g->sc;
    double* nxt = g->sc2;
    for (int k = 0; k < substeps; ++k) {
        a.neighbours = k == 0 ? neighbours : nullptr;
        a.sc = cur;
        a.out = nxt;
        hipLaunchKernelGGL(k_diffuse, dim3(blocks(n, 256)), dim3(256), 0, s, a);
        std::swap(cur, nxt);
    }
    hipLaunchKernelGGL(k_scatter_c, dim3(blocks(n, 256)), dim3(256), 0, s, g->slot, cur, n,
                       state, ld);
    e = hipGetLastError();
    return e == hipSuccess ? ADM1_OK : (int)e;
}

}  // extern "C"
