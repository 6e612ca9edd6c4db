// k_soma.hip -- extracellular substances on gfx950 (paper Sec. 2.1: diffusion of substances as a
// standalone operation once per step; secretion and chemotaxis as agent behaviours) and the
// soma-clustering step built from them (the Sec. 3.4 benchmark).
//
// Field layout: substance s, voxel (i, j, k) at s*V + i + nx*(j + ny*k), binary64, x fastest.
//
//   secrete_count  per agent of type s < 2: one 32-bit atomic increment of its voxel's counter
//   secrete_apply  per agent: exchange its voxel's counter with 0; the one agent that reads the
//                  count m > 0 adds q*m to the voxel (one rounding, whatever the agents' order),
//                  and the counters are zero again for the next step
//   diffuse        one explicit step with decay of both substances, c -> c_next (below)
//   chemotaxis     per agent of type s < 2: gradient of substance s at its voxel by central
//                  differences (closed boundary), move by speed along it
//
// Diffusion is a 7-point stencil, bound by HBM: the algorithmic traffic is one read and one
// write of 8 bytes per voxel.  A workgroup owns a 64 x 16 column of voxels and walks along z:
// each lane keeps the values below, at and above its voxels in registers, so z-neighbours cost
// no loads; x/y-neighbours come from the current plane staged in LDS with a one-voxel halo
// (two buffers, one barrier per plane).  A row of 64 lanes reads 512 contiguous bytes; results
// are stored non-temporally.  The closed boundary is a clamped neighbour index: outside the
// grid the neighbour is the voxel itself and its difference is exactly zero.
#include "kernels.hpp"

namespace bdm {

constexpr int kDiffTX = 64;                 // voxels along x per workgroup (one wavefront row)
constexpr int kDiffTY = 16;                 // voxels along y per workgroup
constexpr int kDiffRows = kDiffTY / 4;      // rows per lane (256 lanes = 64 x 4)

__device__ __forceinline__ int voxel_axis(double v, double origin, double h, int n) {
    double c = floor((v - origin) / h);
    if (!(c >= 0.0)) c = 0.0;  // (also a non-finite position: the grid build flags those)
    if (c > double(n - 1)) c = double(n - 1);
    return int(c);
}

__device__ __forceinline__ int64_t voxel_of(const FieldDev &f, double x, double y, double z) {
    const int i = voxel_axis(x, f.x0, f.h, f.nx);
    const int j = voxel_axis(y, f.y0, f.h, f.ny);
    const int k = voxel_axis(z, f.z0, f.h, f.nz);
    return int64_t(i) + int64_t(f.nx) * (int64_t(j) + int64_t(f.ny) * int64_t(k));
}

__global__ __launch_bounds__(kBlock) void k_secrete_count(const int64_t *n_ptr, int64_t capacity, bdm_soa s,
                                                          FieldDev f, uint32_t *count) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, 0, capacity);
    if (i >= n) return;
    const uint32_t t = s.state[i];
    if (t > 1u) return;
    atomicAdd(&count[int64_t(t) * f.V + voxel_of(f, s.x[i], s.y[i], s.z[i])], 1u);
}

__global__ __launch_bounds__(kBlock) void k_secrete_apply(const int64_t *n_ptr, int64_t capacity, bdm_soa s,
                                                          FieldDev f, uint32_t *count, double *c, double q) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, 0, capacity);
    if (i >= n) return;
    const uint32_t t = s.state[i];
    if (t > 1u) return;
    const int64_t v = int64_t(t) * f.V + voxel_of(f, s.x[i], s.y[i], s.z[i]);
    const uint32_t m = atomicExch(&count[v], 0u);
    if (m != 0u) c[v] = c[v] + q * double(m);
}

__global__ __launch_bounds__(kBlock) void k_diffuse(FieldDev f, const double *__restrict__ cin,
                                                    double *__restrict__ cout, double lam, double kdec,
                                                    int32_t zchunk, int32_t nzc) {
    __shared__ double s_pl[2][kDiffTY + 2][kDiffTX + 2];
    const int tx = int(threadIdx.x & 63), ty = int(threadIdx.x >> 6);
    const int xb = int(blockIdx.x) * kDiffTX, yb = int(blockIdx.y) * kDiffTY;
    const int sub = int(blockIdx.z) / nzc, zc = int(blockIdx.z) % nzc;
    const int zb = zc * zchunk;
    const int ze = min(f.nz, zb + zchunk);
    const double *in = cin + int64_t(sub) * f.V;
    double *out = cout + int64_t(sub) * f.V;
    const int nx = f.nx, ny = f.ny, nz = f.nz;
    const int64_t plane = int64_t(nx) * ny;
    const int x = xb + tx;
    const int xc = min(x, nx - 1);                  // lanes past the edge mirror the last voxel
    const int xl = max(xb - 1, 0), xr = min(xb + kDiffTX, nx - 1);  // halo columns (clamped)
    int64_t rowoff[kDiffRows];
    int yr[kDiffRows];
#pragma unroll
    for (int r = 0; r < kDiffRows; ++r) {
        yr[r] = yb + ty + 4 * r;
        rowoff[r] = int64_t(min(yr[r], ny - 1)) * nx;
    }
    // y-halo rows (clamped): wavefront 0 stages the row below the tile, wavefront 1 the row above
    const int yh = ty == 0 ? max(yb - 1, 0) : min(yb + kDiffTY, ny - 1);
    const int hrow = ty == 0 ? 0 : kDiffTY + 1;
    double below[kDiffRows], cur[kDiffRows], above[kDiffRows];
    const int64_t zoff0 = int64_t(zb) * plane, zoffm = int64_t(max(zb - 1, 0)) * plane;
#pragma unroll
    for (int r = 0; r < kDiffRows; ++r) {
        cur[r] = in[zoff0 + rowoff[r] + xc];
        below[r] = in[zoffm + rowoff[r] + xc];
    }
    for (int z = zb; z < ze; ++z) {
        const int64_t zoff = int64_t(z) * plane;
        const int64_t zoffp = int64_t(min(z + 1, nz - 1)) * plane;
        const int b = (z - zb) & 1;
#pragma unroll
        for (int r = 0; r < kDiffRows; ++r) {
            above[r] = in[zoffp + rowoff[r] + xc];
            s_pl[b][1 + ty + 4 * r][1 + tx] = cur[r];
        }
        if (ty < 2) s_pl[b][hrow][1 + tx] = in[zoff + int64_t(yh) * nx + xc];
        if (tx < 2 * kDiffRows) {
            // x-halo: lanes 0..3 the left column, lanes 4..7 the right column, 4 rows per wave
            const int r = tx % kDiffRows;
            const int col = tx < kDiffRows ? xl : xr;
            s_pl[b][1 + ty + 4 * r][tx < kDiffRows ? 0 : kDiffTX + 1] = in[zoff + rowoff[r] + col];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kDiffRows; ++r) {
            const int row = 1 + ty + 4 * r;
            const double c = cur[r];
            const double xm = s_pl[b][row][tx], xp = s_pl[b][row][tx + 2];
            const double ym = s_pl[b][row - 1][tx + 1], yp = s_pl[b][row + 1][tx + 1];
            const double lap = (((xm - c) + (xp - c)) + ((ym - c) + (yp - c))) + ((below[r] - c) + (above[r] - c));
            if (x < nx && yr[r] < ny)  // streamed out: the next read is a whole field later
                __builtin_nontemporal_store(c + (lam * lap - kdec * c), &out[zoff + int64_t(yr[r]) * nx + x]);
            below[r] = c;
            cur[r] = above[r];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_chemotaxis(const int64_t *n_ptr, int64_t capacity, bdm_soa s,
                                                       FieldDev f, const double *__restrict__ c, double speed) {
    const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, 0, capacity);
    if (a >= n) return;
    const uint32_t t = s.state[a];
    if (t > 1u) return;
    const double px = s.x[a], py = s.y[a], pz = s.z[a];
    const int i = voxel_axis(px, f.x0, f.h, f.nx);
    const int j = voxel_axis(py, f.y0, f.h, f.ny);
    const int k = voxel_axis(pz, f.z0, f.h, f.nz);
    const double *cs = c + int64_t(t) * f.V;
    const int64_t row = int64_t(f.nx), plane = int64_t(f.nx) * f.ny;
    const int64_t v = int64_t(i) + row * j + plane * k;
    const double gx = cs[v - i + min(i + 1, f.nx - 1)] - cs[v - i + max(i - 1, 0)];
    const double gy = cs[v + row * (min(j + 1, f.ny - 1) - j)] - cs[v + row * (max(j - 1, 0) - j)];
    const double gz = cs[v + plane * (min(k + 1, f.nz - 1) - k)] - cs[v + plane * (max(k - 1, 0) - k)];
    const double g2 = (gx * gx + gy * gy) + gz * gz;
    if (!(g2 > 0.0)) return;
    const double sc = speed / __builtin_sqrt(g2);
    s.x[a] = px + sc * gx;
    s.y[a] = py + sc * gy;
    s.z[a] = pz + sc * gz;
}

__global__ __launch_bounds__(kBlock) void k_field_fill(double *c, uint32_t *count, int64_t len) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; v < len; v += stride) {
        c[v] = 0.0;
        count[v] = 0u;
    }
}

static unsigned agent_blocks(int64_t capacity) {
    const int64_t b = (capacity + kBlock - 1) / kBlock;
    return unsigned(b < 1 ? 1 : b);
}

void diffusion_launch_shape(const FieldDev &f, int32_t *zchunk, int32_t *nzc, dim3 *grid) {
    const int64_t tiles = int64_t((f.nx + kDiffTX - 1) / kDiffTX) * ((f.ny + kDiffTY - 1) / kDiffTY);
    // about 8192 workgroups (32 per CU: the latency of the plane loads is hidden by many
    // workgroups in flight rather than by long z runs), at least 8 planes per chunk, at most
    // 32767 chunks per substance
    int64_t want = (8192 + 2 * tiles - 1) / (2 * tiles);
    if (want < 1) want = 1;
    int64_t zc = (f.nz + want - 1) / want;
    if (zc < 8) zc = 8;
    const int64_t minzc = (f.nz + 32766) / 32767;
    if (zc < minzc) zc = minzc;
    *zchunk = int32_t(zc);
    *nzc = int32_t((f.nz + zc - 1) / zc);
    *grid = dim3(unsigned((f.nx + kDiffTX - 1) / kDiffTX), unsigned((f.ny + kDiffTY - 1) / kDiffTY),
                 unsigned(2 * *nzc));
}

void launch_diffuse(const FieldDev &f, const double *cin, double *cout, double lam, double kdec, hipStream_t st) {
    int32_t zchunk = 0, nzc = 0;
    dim3 grid;
    diffusion_launch_shape(f, &zchunk, &nzc, &grid);
    hipLaunchKernelGGL(k_diffuse, grid, dim3(kBlock), 0, st, f, cin, cout, lam, kdec, zchunk, nzc);
}

void launch_secrete(const bdm_soa &s, int64_t capacity, const FieldDev &f, uint32_t *count, double *c, double q,
                    hipStream_t st) {
    const unsigned nb = agent_blocks(capacity);
    hipLaunchKernelGGL(k_secrete_count, dim3(nb), dim3(kBlock), 0, st, s.n, capacity, s, f, count);
    hipLaunchKernelGGL(k_secrete_apply, dim3(nb), dim3(kBlock), 0, st, s.n, capacity, s, f, count, c, q);
}

void launch_chemotaxis(const bdm_soa &s, int64_t capacity, const FieldDev &f, const double *c, double speed,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_chemotaxis, dim3(agent_blocks(capacity)), dim3(kBlock), 0, st, s.n, capacity, s, f, c,
                       speed);
}

void launch_field_fill(double *c, uint32_t *count, int64_t len, hipStream_t st) {
    int64_t nb = (len + kBlock - 1) / kBlock;
    if (nb > 16384) nb = 16384;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_field_fill, dim3(unsigned(nb)), dim3(kBlock), 0, st, c, count, len);
}

}  // namespace bdm
