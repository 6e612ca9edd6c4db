// k_geom.hip -- mechanics of spheres and cylinders (neurite elements) on gfx950 (paper Sec. 2.2:
// a neurite element is a cylinder with a point mass at its distal end; Sec. 2.1: agents interact
// with the agents of the 27 boxes around their own).
//
// A cylinder agent's position is its distal end q; its proximal end p and diameter dc are kept
// by agent id.  Its grid diameter is 2|q - p| + dc (the sphere about q holding the whole body),
// so a grid whose box edge is the largest grid diameter finds every contact in the 27 boxes.
//
//   reach  per agent: a cylinder's grid diameter from its current ends
//   grid   the sphere path's build (keys, sort, starts) on the grid diameters
//   mid    per sorted agent, the binary32 sphere about its body's midpoint that holds the body
//   geom   one lane per box-sorted agent walks the 27 boxes as 9 key runs; a candidate passes a
//          conservative binary32 test of the two midpoint spheres, then the closest points
//          of the two axes carry virtual spheres of the bodies' diameters and the sphere law
//          acts between them; a cylinder takes the share s of the force (s its closest point's
//          position along p -> q); gate, clamp and move as the sphere step (a cylinder moves its
//          distal end)
//
// The arithmetic follows the same expressions in the same order as the definition, so results
// are reproducible bit for bit.  The walk visits many candidates: the grid sphere about the
// distal end (radius l + d/2) sets a box edge of up to twice a cylinder's length, about 330
// candidates per agent at the neurite workload's 18 um boxes.  The midpoint spheres, half as
// wide for a cylinder, pass far fewer of them to the closest-point law, which runs over per-lane
// queues in walk order (the order of the sums is the walk's).
#include "kernels.hpp"

namespace bdm {

__device__ __forceinline__ double dot3(double ax, double ay, double az, double bx, double by, double bz) {
    return (ax * bx + ay * by) + az * bz;
}

__device__ __forceinline__ double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

// Closest point of segment p -> q to c: parameter in [0, 1]; 1 for a segment of length 0.
__device__ __forceinline__ double seg_point(double px, double py, double pz, double qx, double qy, double qz,
                                            double cx, double cy, double cz) {
    const double dx = qx - px, dy = qy - py, dz = qz - pz;
    const double a = dot3(dx, dy, dz, dx, dy, dz);
    if (!(a > 0.0)) return 1.0;
    return clamp01(dot3(cx - px, cy - py, cz - pz, dx, dy, dz) / a);
}

// Closest points of segments p1 -> q1 and p2 -> q2 (parameters s, t): the clamped stationary
// point of the squared distance, t re-clamped and s recomputed at a clamped t; near-parallel
// segments (a e - b^2 <= 2^-40 a e) start from s = 0; a segment of length 0 is its distal end.
__device__ __forceinline__ void seg_seg(const double p1[3], const double q1[3], const double p2[3],
                                        const double q2[3], double &s, double &t) {
    const double d1x = q1[0] - p1[0], d1y = q1[1] - p1[1], d1z = q1[2] - p1[2];
    const double d2x = q2[0] - p2[0], d2y = q2[1] - p2[1], d2z = q2[2] - p2[2];
    const double rx = p1[0] - p2[0], ry = p1[1] - p2[1], rz = p1[2] - p2[2];
    const double a = dot3(d1x, d1y, d1z, d1x, d1y, d1z), e = dot3(d2x, d2y, d2z, d2x, d2y, d2z);
    const double f = dot3(d2x, d2y, d2z, rx, ry, rz);
    if (!(a > 0.0) && !(e > 0.0)) {
        s = 1.0;
        t = 1.0;
    } else if (!(a > 0.0)) {
        s = 1.0;
        t = clamp01(f / e);
    } else {
        const double c = dot3(d1x, d1y, d1z, rx, ry, rz);
        if (!(e > 0.0)) {
            t = 1.0;
            s = clamp01(-c / a);
        } else {
            const double b = dot3(d1x, d1y, d1z, d2x, d2y, d2z);
            const double ae = a * e;
            const double denom = ae - b * b;
            s = denom > 0x1.0p-40 * ae ? clamp01((b * f - c * e) / denom) : 0.0;
            const double tn = b * s + f;
            if (tn < 0.0) {
                t = 0.0;
                s = clamp01(-c / a);
            } else if (tn > e) {
                t = 1.0;
                s = clamp01((b - c) / a);
            } else {
                t = tn / e;
            }
        }
    }
}

struct Body {
    double x[3];   // centre, or distal end
    double p[3];   // proximal end (cylinders)
    double d;      // sphere diameter, or cylinder diameter
    bool cyl;
};

// Sphere law between virtual spheres (ci, Di) and (cj, Dj): force on i into f; true on contact.
__device__ __forceinline__ bool sphere_law(const double ci[3], double Di, const double cj[3], double Dj, double k,
                                           double gamma, double f[3]) {
    f[0] = f[1] = f[2] = 0.0;
    const double dx = ci[0] - cj[0], dy = ci[1] - cj[1], dz = ci[2] - cj[2];
    const double dist = __builtin_sqrt((dx * dx + dy * dy) + dz * dz);
    const double ri = 0.5 * Di, rj = 0.5 * Dj;
    const double delta = (ri + rj) - dist;
    if (!(delta > 0.0)) return false;
    if (dist == 0.0) return true;
    const double rhat = (ri * rj) / (ri + rj);
    const double F = k * delta - gamma * __builtin_sqrt(rhat * delta);
    const double sc = F / dist;
    f[0] = sc * dx;
    f[1] = sc * dy;
    f[2] = sc * dz;
    return true;
}

__device__ __forceinline__ bool body_pair(const Body &bi, const Body &bj, double k, double gamma, double f[3]) {
    double ci[3], cj[3], share = 1.0;
    if (bi.cyl && bj.cyl) {
        double s, t;
        seg_seg(bi.p, bi.x, bj.p, bj.x, s, t);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ci[a] = bi.p[a] + s * (bi.x[a] - bi.p[a]);
            cj[a] = bj.p[a] + t * (bj.x[a] - bj.p[a]);
        }
        share = s;
    } else if (bi.cyl) {
        const double s = seg_point(bi.p[0], bi.p[1], bi.p[2], bi.x[0], bi.x[1], bi.x[2], bj.x[0], bj.x[1], bj.x[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ci[a] = bi.p[a] + s * (bi.x[a] - bi.p[a]);
            cj[a] = bj.x[a];
        }
        share = s;
    } else if (bj.cyl) {
        const double t = seg_point(bj.p[0], bj.p[1], bj.p[2], bj.x[0], bj.x[1], bj.x[2], bi.x[0], bi.x[1], bi.x[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ci[a] = bi.x[a];
            cj[a] = bj.p[a] + t * (bj.x[a] - bj.p[a]);
        }
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ci[a] = bi.x[a];
            cj[a] = bj.x[a];
        }
    }
    const bool hit = sphere_law(ci, bi.d, cj, bj.d, k, gamma, f);
    f[0] = share * f[0];
    f[1] = share * f[1];
    f[2] = share * f[2];
    return hit;
}

__device__ __forceinline__ Body load_body(const double4 &r, uint8_t kind, uint32_t id, const CylIn &cyl) {
    Body b;
    b.x[0] = r.x;
    b.x[1] = r.y;
    b.x[2] = r.z;
    b.cyl = kind == 1;
    if (b.cyl) {
        b.p[0] = cyl.px[id];
        b.p[1] = cyl.py[id];
        b.p[2] = cyl.pz[id];
        b.d = cyl.dc[id];
    } else {
        b.p[0] = r.x;
        b.p[1] = r.y;
        b.p[2] = r.z;
        b.d = 2.0 * r.w;  // the sorted record holds d/2; doubling is exact
    }
    return b;
}

__global__ __launch_bounds__(kBlock) void k_geom_reach(const int64_t *n_ptr, int64_t capacity, bdm_soa s, CylIn cyl) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n = live_count(n_ptr, 0, capacity);
    if (i >= n || s.state[i] != 1) return;
    const uint32_t id = s.id[i];
    if (int64_t(id) >= capacity) return;  // ids index the caller's cylinder arrays
    const double dx = s.x[i] - cyl.px[id], dy = s.y[i] - cyl.py[id], dz = s.z[i] - cyl.pz[id];
    s.diam[i] = 2.0 * __builtin_sqrt(dot3(dx, dy, dz, dx, dy, dz)) + cyl.dc[id];
}

constexpr int kGeomQueue = 16;  // candidates past the bounding-sphere test a lane holds (16 KB of LDS per workgroup)

// The walk's filter records, one per sorted agent: the sphere about the body's midpoint that
// holds the whole body (half its length plus half its diameter; a sphere is its own), as the
// binary32 copy of the crowded sphere kernel: relative to the lattice origin, the radius scaled
// by kPretestRadius, tested with pretest_slack.  A contact's closest points lie on the two axes,
// each within half its axis of the midpoint, and their distance is below the sum of the half
// diameters, so the midpoint spheres of a contact overlap; their radii sum to at most the
// largest grid diameter (twice a length plus a diameter), the box edge, which the slack assumes.
// The grid sphere about the distal end, which the box search needs, has about twice the radius.
__global__ __launch_bounds__(kBlock) void k_geom_mid(const GridDev *__restrict__ g, const double4 *__restrict__ pos4,
                                                     const uint32_t *__restrict__ id_s,
                                                     const uint8_t *__restrict__ state_s, CylIn cyl, int64_t capacity,
                                                     float4 *__restrict__ mid) {
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (!g->valid || s >= g->n) return;
    const double4 r = pos4[s];
    double mx = r.x, my = r.y, mz = r.z, rad = r.w;  // a sphere: its centre and radius
    const uint32_t id = id_s[s];
    if (state_s[s] == 1 && int64_t(id) < capacity) {
        const double px = cyl.px[id], py = cyl.py[id], pz = cyl.pz[id];
        const double dx = r.x - px, dy = r.y - py, dz = r.z - pz;
        mx = 0.5 * (px + r.x);
        my = 0.5 * (py + r.y);
        mz = 0.5 * (pz + r.z);
        rad = 0.5 * __builtin_sqrt(dot3(dx, dy, dz, dx, dy, dz)) + 0.5 * cyl.dc[id];
    }
    mid[s] = make_float4(float(mx - double(g->cmin[0]) * g->b), float(my - double(g->cmin[1]) * g->b),
                         float(mz - double(g->cmin[2]) * g->b), float(rad * kPretestRadius));
}

// Six wavefronts per SIMD (80 registers, a few spilled) instead of the four that the
// compiler's 102 registers allow: measured 2.02 -> 1.95 ms per step of the neurite workload.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_geom(GridDev *__restrict__ g, const double4 *__restrict__ pos4,
                                                 const double *__restrict__ adh_s, const uint32_t *__restrict__ id_s,
                                                 const uint8_t *__restrict__ state_s,
                                                 const uint32_t *__restrict__ start, CylIn cyl, GeomArgs a,
                                                 bdm_soa out, uint32_t *counts, const float4 *__restrict__ mid) {
    __shared__ uint32_t s_q[kGeomQueue][kBlock];  // each lane uses its own column only
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (!g->valid || s >= g->n) return;
    const double4 ri = pos4[s];
    const uint32_t idi = id_s[s];
    const uint8_t ki = state_s[s];
    if (ki == 1 && int64_t(idi) >= a.capacity) {
        atomicOr(&g->flags, BDM_FLAG_BADID);
        return;
    }
    const Body bi = load_body(ri, ki, idi, cyl);
    const double b = g->b;
    const int cx = box_coord(ri.x, b, g->cmin[0], g->dims[0], false);
    const int cy = box_coord(ri.y, b, g->cmin[1], g->dims[1], false);
    const int cz = box_coord(ri.z, b, g->cmin[2], g->dims[2], false);
    const int nx = g->dims[0], ny = g->dims[1], nz = g->dims[2];
    const float4 mi = mid[s];
    const float slack = pretest_slack(g);
    double sx = 0.0, sy = 0.0, sz = 0.0;
    uint32_t contacts = 0;
    // Candidates that pass the bounding-sphere test go to the lane's queue in walk order; the
    // closest-point law runs over the queues when one fills and at the end.  Run inside the walk,
    // it cost every lane of the wavefront a pair evaluation at nearly every candidate (some
    // lane almost always passes); over the queues it runs as often as the longest queue.
    uint32_t qn = 0;
    const int t = threadIdx.x;
    auto flush = [&]() {
        for (uint32_t k = 0; k < qn; ++k) {
            const uint32_t j = s_q[k][t];
            const double4 rj = pos4[j];
            const uint8_t kj = state_s[j];
            const uint32_t idj = id_s[j];
            if (kj == 1 && int64_t(idj) >= a.capacity) continue;
            const Body bj = load_body(rj, kj, idj, cyl);
            double f[3];
            if (body_pair(bi, bj, a.k, a.gamma, f)) {
                ++contacts;
                sx = sx + f[0];
                sy = sy + f[1];
                sz = sz + f[2];
            }
        }
        qn = 0;
    };
    for (int r = 0; r < 9; ++r) {
        const int zz = cz + r / 3 - 1, yy = cy + r % 3 - 1;
        if (zz < 0 || zz >= nz || yy < 0 || yy >= ny) continue;
        const int x0 = cx > 0 ? cx - 1 : 0, x1 = cx < nx - 1 ? cx + 1 : nx - 1;
        const uint32_t kb = uint32_t(x0) + uint32_t(nx) * (uint32_t(yy) + uint32_t(ny) * uint32_t(zz));
        const uint32_t lo = start[kb] & kStartMask, hi = start[kb + uint32_t(x1 - x0) + 1u] & kStartMask;
        for (uint32_t j = lo; j < hi; ++j) {
            if (j == uint32_t(s)) continue;
            s_q[qn][t] = j;
            qn += maybe_touch(mi, mid[j], slack) ? 1u : 0u;
            if (__any(qn == uint32_t(kGeomQueue))) flush();  // (the wavefront together)
        }
    }
    flush();
    // gate, clamp and move (the sphere step's rules)
    double nxp = ri.x, nyp = ri.y, nzp = ri.z;
    const double fnorm = __builtin_sqrt((sx * sx + sy * sy) + sz * sz);
    if (!(fnorm < adh_s[s])) {
        double ux = a.dt * sx, uy = a.dt * sy, uz = a.dt * sz;
        const double len = __builtin_sqrt((ux * ux + uy * uy) + uz * uz);
        if (len > a.max_disp) {
            const double scale = a.max_disp / len;
            ux = ux * scale;
            uy = uy * scale;
            uz = uz * scale;
        }
        nxp = ri.x + ux;
        nyp = ri.y + uy;
        nzp = ri.z + uz;
    }
    out.x[s] = nxp;
    out.y[s] = nyp;
    out.z[s] = nzp;
    out.diam[s] = 2.0 * ri.w;
    out.adh[s] = adh_s[s];
    out.id[s] = idi;
    out.state[s] = ki;
    if (out.fx) out.fx[s] = sx;
    if (out.fy) out.fy[s] = sy;
    if (out.fz) out.fz[s] = sz;
    if (counts) counts[s] = contacts;
}

void launch_geom_reach(const bdm_soa &s, int64_t capacity, const CylIn &cyl, hipStream_t st) {
    int64_t nb = (capacity + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_geom_reach, dim3(unsigned(nb)), dim3(kBlock), 0, st, s.n, capacity, s, cyl);
}

void launch_geom(const bdm_soa &s, const CylIn &cyl, const GeomArgs &a, const Ws &w, uint32_t *counts,
                 hipStream_t st) {
    int64_t nb = (a.capacity + kBlock - 1) / kBlock;
    if (nb < 1) nb = 1;
    // the filter records go to the binary32 copy's array (the sphere build leaves it unused)
    hipLaunchKernelGGL(k_geom_mid, dim3(unsigned(nb)), dim3(kBlock), 0, st, &w.grid[0], w.pos4, w.ids, w.state, cyl,
                       a.capacity, w.pos4f);
    hipLaunchKernelGGL(k_geom, dim3(unsigned(nb)), dim3(kBlock), 0, st, &w.grid[0], w.pos4, w.adh, w.ids, w.state,
                       w.start, cyl, a, s, counts, w.pos4f);
}

}  // namespace bdm
