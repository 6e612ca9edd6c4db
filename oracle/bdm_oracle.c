/*
 * bdm_oracle.c -- plain, single-threaded FP64 CPU reference ("the oracle") for the
 * mechanical-interaction hot path of the BioDynaMo agent-based engine
 * (Breitwieser et al., arXiv 2006.06775).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library.  The GPU library never links, includes or calls it, and
 * it shares no source with the GPU path.  Everything here is written for a reader to check
 * against the paper by eye: no blocking, fusion or reordering beyond what the method states.
 *
 * What is computed (paper sections in brackets):
 *   - Uniform grid environment [Sec. 2.1, "Simulation concepts"]: space is cut into equal cubic
 *     boxes, an agent belongs to the box holding its centre, its environment is its own box plus
 *     the 26 around it, and the box edge follows the largest agent.
 *   - Mechanical force between agent pairs as an agent operation run every step [Sec. 2.1];
 *     the model is the Zubler & Douglas / Cortex3D one [Sec. 1 and Sec. 3.4].  The sphere-sphere
 *     law used is F = k*delta - gamma*sqrt(rhat*delta) on overlap delta, rhat = ri*rj/(ri+rj).
 *   - Adherence-gated, clamped explicit displacement of each agent from its summed force.
 *   - Tumour-spheroid growth and division [Sec. 3.2] and the SIR epidemic model [Sec. 3.3:
 *     infection within a radius with a probability, recovery with a probability each step,
 *     bounded random movement], both on the same grid.
 *   - Tumour-spheroid apoptosis and Brownian migration, and the convex-hull diameter (in the
 *     Python wrapper) [Sec. 3.2].
 *   - Extracellular substances [Sec. 2.1]: an explicit diffusion step with decay on a voxel grid
 *     (a standalone operation), secretion and chemotaxis (agent behaviours), and the soma-
 *     clustering model built from them [Sec. 3.4 benchmark].
 *   - Cylinder geometry of neurite elements [Sec. 2.2]: sphere-cylinder and cylinder-cylinder
 *     contacts through the closest points of the bodies' axes, on the same grid.
 *   - Counter-based Philox4x64-10 random numbers (Salmon, Moraes, Dror, Shaw, SC'11).
 *
 * Where the paper is silent the readings are fixed as follows (each one is restated at the
 * function that applies it):
 *   force sign        F > 0 repels: F_i += (F/dist) * (x_i - x_j)
 *   contact           delta = (ri + rj) - dist > 0, strictly; coincident centres add nothing
 *   mobility          unit mass: displacement = dt * F_i
 *   adherence gate    |F_i| < adh_i -> no movement (equality moves)
 *   clamp             |disp| > max_disp -> disp *= max_disp / |disp|
 *   update            synchronous: every force from positions at t, then every position at t+1
 *   box edge          b = max diameter (or an explicit box >= it); lattice c = floor(x / b);
 *                     origin/dims from min/max c; key = cx + nx*(cy + ny*cz)
 *   order in a box    ascending agent id; forces are summed over candidates in ascending
 *                     (key, id) order starting from +0.0
 *   arithmetic        IEEE binary64, no contraction (built with -ffp-contract=off)
 *
 * Agents are stored in id order: the array index IS the agent id.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_ENOMEM = -2,
    ORC_ENONFINITE = -3,
    ORC_ETOOMANYBOXES = -4,
};

/* ------------------------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11, "Parallel random numbers: as easy as 1, 2, 3").          */
/* Ten rounds of: two 64x64->128 multiplications of counter words 0 and 2 by the round           */
/* multipliers, outputs recombined with counter words 1, 3 and the key; the key is bumped by the */
/* Weyl constants between rounds.                                                                */
/* ------------------------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL
#define PHILOX_W1 0xBB67AE8584CAA73BULL

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Purposes of random draws: word 0 of the counter is purpose + (attempt << 8). */
enum { RNG_INIT = 1, RNG_MOVE = 2, RNG_REC = 3, RNG_INF = 4, RNG_DIV = 5, RNG_APO = 6, RNG_MIG = 7 };

/* One Philox block keyed by (seed, salt) at counter (purpose + attempt*2^8, id, step, 0). */
void orc_draw(uint64_t seed, uint64_t salt, uint64_t purpose, uint64_t attempt, uint64_t id,
              uint64_t step, uint64_t out[4])
{
    uint64_t ctr[4] = {purpose + (attempt << 8), id, step, 0};
    uint64_t key[2] = {seed, salt};
    orc_philox4x64_10(ctr, key, out);
}

/* Uniform double in [0, 1): the top 53 bits of a word times 2^-53 (exact). */
double orc_u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

/* Bernoulli(p) from one word: true iff w < floor(p * 2^64); p <= 0 never, p >= 1 always. */
int orc_bernoulli(uint64_t w, double p)
{
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return 1;
    uint64_t threshold = (uint64_t)ldexp(p, 64); /* exact scaling; conversion truncates = floor */
    return w < threshold;
}

/* ------------------------------------------------------------------------------------------ */
/* Seeded generators of the initial agent state                                               */
/* ------------------------------------------------------------------------------------------ */

/* Agents uniform in the cube [0, L)^3, diameters uniform in [dmin, dmax), one adherence value.
 * Agent id draws one block at (INIT, attempt 0, id, step 0): words 0..2 -> x, y, z, word 3 -> d. */
int orc_generate_cube(int64_t n, uint64_t seed, uint64_t salt, double L, double dmin, double dmax,
                      double adh, double *x, double *y, double *z, double *d, double *a)
{
    if (n < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t w[4];
        orc_draw(seed, salt, RNG_INIT, 0, (uint64_t)i, 0, w);
        x[i] = L * orc_u01(w[0]);
        y[i] = L * orc_u01(w[1]);
        z[i] = L * orc_u01(w[2]);
        if (d) d[i] = dmin + (dmax - dmin) * orc_u01(w[3]);
        if (a) a[i] = adh;
    }
    return ORC_OK;
}

/* Agents uniform in the ball of radius R about the origin, by rejection from the cube
 * [-R, R)^3: attempt t draws (INIT, t, id, 0); v = 2u - 1 per axis from words 0..2; accept when
 * |v|^2 <= 1 and place the agent at R*v.  The accepted block's word 3 sets the diameter uniform
 * in [dlo, dhi).  After 64 rejected attempts the agent sits at the origin. */
int orc_generate_ball(int64_t n, uint64_t seed, uint64_t salt, double R, double dlo, double dhi,
                      double adh, double *x, double *y, double *z, double *d, double *a)
{
    if (n < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        double px = 0.0, py = 0.0, pz = 0.0, u3 = 0.0;
        for (uint64_t attempt = 0; attempt < 64; ++attempt) {
            uint64_t w[4];
            orc_draw(seed, salt, RNG_INIT, attempt, (uint64_t)i, 0, w);
            double vx = 2.0 * orc_u01(w[0]) - 1.0;
            double vy = 2.0 * orc_u01(w[1]) - 1.0;
            double vz = 2.0 * orc_u01(w[2]) - 1.0;
            double s = (vx * vx + vy * vy) + vz * vz;
            if (s <= 1.0) {
                px = R * vx; py = R * vy; pz = R * vz;
                u3 = orc_u01(w[3]);
                break;
            }
        }
        x[i] = px; y[i] = py; z[i] = pz;
        if (d) d[i] = dlo + (dhi - dlo) * u3;
        if (a) a[i] = adh;
    }
    return ORC_OK;
}

/* SIR population: points uniform in [0, L)^3 as in the cube generator; the agents with
 * id < n_infected start infected (1), all others susceptible (0). */
int orc_generate_sir(int64_t n, uint64_t seed, uint64_t salt, double L, int64_t n_infected,
                     double *x, double *y, double *z, uint8_t *state)
{
    if (n < 0 || n_infected < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t w[4];
        orc_draw(seed, salt, RNG_INIT, 0, (uint64_t)i, 0, w);
        x[i] = L * orc_u01(w[0]);
        y[i] = L * orc_u01(w[1]);
        z[i] = L * orc_u01(w[2]);
        state[i] = (i < n_infected) ? 1 : 0;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Uniform grid [Sec. 2.1]                                                                    */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    double b;          /* box edge */
    int32_t periodic;  /* 0: open space; 1: periodic cube [0, L)^3 */
    double L;
    int64_t cmin[3];   /* lattice coordinate of box 0 (open space) */
    int64_t dims[3];   /* boxes per axis */
    int64_t nboxes;
} orc_grid;

static int finite3(double a, double b, double c) { return isfinite(a) && isfinite(b) && isfinite(c); }

/* Box edge and lattice.  Open space: b = explicit box (must be >= the largest diameter) or the
 * largest diameter itself ("box size chosen based on the largest agent"); lattice coordinate
 * c = floor(x / b) per axis; box 0 sits at the minimum c over agents, dims = max c - min c + 1.
 * Periodic cube of edge L: nb = floor(L / box) boxes per axis (at least 3), b = L / nb. */
int orc_grid_setup(int64_t n, const double *x, const double *y, const double *z, const double *d,
                   double box, int32_t periodic, double L, int64_t max_boxes, orc_grid *g)
{
    memset(g, 0, sizeof *g);
    g->periodic = periodic;
    g->L = L;
    double dmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!finite3(x[i], y[i], z[i])) return ORC_ENONFINITE;
        if (d) {
            if (!isfinite(d[i])) return ORC_ENONFINITE;
            if (d[i] > dmax) dmax = d[i];
        }
    }
    if (periodic) {
        if (!(L > 0.0) || !(box > 0.0) || box < dmax) return ORC_EINVAL;
        double nb = floor(L / box);
        if (nb < 3.0) return ORC_EINVAL;
        g->b = L / nb;
        for (int a = 0; a < 3; ++a) { g->cmin[a] = 0; g->dims[a] = (int64_t)nb; }
    } else {
        if (box > 0.0) {
            if (box < dmax) return ORC_EINVAL;
            g->b = box;
        } else {
            g->b = dmax;
        }
        if (n == 0) { g->nboxes = 0; return ORC_OK; }
        if (!(g->b > 0.0)) return ORC_EINVAL;
        int64_t lo[3], hi[3];
        for (int64_t i = 0; i < n; ++i) {
            int64_t c[3] = {(int64_t)floor(x[i] / g->b), (int64_t)floor(y[i] / g->b),
                            (int64_t)floor(z[i] / g->b)};
            for (int a = 0; a < 3; ++a) {
                if (i == 0 || c[a] < lo[a]) lo[a] = c[a];
                if (i == 0 || c[a] > hi[a]) hi[a] = c[a];
            }
        }
        for (int a = 0; a < 3; ++a) { g->cmin[a] = lo[a]; g->dims[a] = hi[a] - lo[a] + 1; }
    }
    double total = (double)g->dims[0] * (double)g->dims[1] * (double)g->dims[2];
    if (total > (double)max_boxes) return ORC_ETOOMANYBOXES;
    g->nboxes = g->dims[0] * g->dims[1] * g->dims[2];
    return ORC_OK;
}

/* Box coordinate of a position along one axis. */
static int64_t box_coord(const orc_grid *g, double v, int axis)
{
    int64_t c = (int64_t)floor(v / g->b);
    if (g->periodic) {
        if (c < 0) c = 0;
        if (c > g->dims[axis] - 1) c = g->dims[axis] - 1;
        return c;
    }
    return c - g->cmin[axis];
}

static int64_t box_key(const orc_grid *g, int64_t cx, int64_t cy, int64_t cz)
{
    return cx + g->dims[0] * (cy + g->dims[1] * cz);
}

/* Keys, box-sorted order and box start offsets.  order[] lists agent ids sorted by (key, id):
 * a stable counting sort over ids.  start[k] is the first position of box k in order[];
 * start[nboxes] = n. */
int orc_grid_sort(int64_t n, const double *x, const double *y, const double *z, const orc_grid *g,
                  uint32_t *key, uint32_t *order, uint32_t *start)
{
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = box_coord(g, x[i], 0), cy = box_coord(g, y[i], 1), cz = box_coord(g, z[i], 2);
        key[i] = (uint32_t)box_key(g, cx, cy, cz);
    }
    for (int64_t k = 0; k <= g->nboxes; ++k) start[k] = 0;
    for (int64_t i = 0; i < n; ++i) start[key[i] + 1] += 1;
    for (int64_t k = 0; k < g->nboxes; ++k) start[k + 1] += start[k];
    uint32_t *cursor = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g->nboxes + 1));
    if (!cursor) return ORC_ENOMEM;
    memcpy(cursor, start, sizeof(uint32_t) * (size_t)(g->nboxes + 1));
    for (int64_t i = 0; i < n; ++i) order[cursor[key[i]]++] = (uint32_t)i;
    free(cursor);
    return ORC_OK;
}

/* Box key of the neighbour box at offset (ox, oy, oz) from box (cx, cy, cz), or -1 when it lies
 * outside an open grid.  Periodic grids wrap each axis modulo the box count. */
static int64_t neighbour_key(const orc_grid *g, int64_t cx, int64_t cy, int64_t cz, int ox, int oy,
                             int oz)
{
    int64_t c[3] = {cx + ox, cy + oy, cz + oz};
    for (int a = 0; a < 3; ++a) {
        if (g->periodic) {
            c[a] = (c[a] + g->dims[a]) % g->dims[a];
        } else if (c[a] < 0 || c[a] >= g->dims[a]) {
            return -1;
        }
    }
    return box_key(g, c[0], c[1], c[2]);
}

/* ------------------------------------------------------------------------------------------ */
/* Sphere-sphere force and displacement                                                       */
/* ------------------------------------------------------------------------------------------ */

/* Force on sphere i from sphere j (binary64).  dx = x_i - x_j, dist = |dx|, ri = di/2,
 * delta = (ri + rj) - dist.  No contact unless delta > 0.  rhat = (ri*rj)/(ri+rj),
 * F = k*delta - gamma*sqrt(rhat*delta), and the pair adds (F/dist)*dx to F_i (nothing when the
 * centres coincide).  Returns 1 on contact. */
int orc_pair_force_f64(double xi, double yi, double zi, double di, double xj, double yj, double zj,
                       double dj, double k, double gamma, double out[3])
{
    out[0] = 0.0; out[1] = 0.0; out[2] = 0.0;
    double dx = xi - xj, dy = yi - yj, dz = zi - zj;
    double dist = sqrt((dx * dx + dy * dy) + dz * dz);
    double ri = 0.5 * di, rj = 0.5 * dj;
    double delta = (ri + rj) - dist;
    if (!(delta > 0.0)) return 0;
    if (dist == 0.0) return 1;
    double rhat = (ri * rj) / (ri + rj);
    double F = k * delta - gamma * sqrt(rhat * delta);
    double s = F / dist;
    out[0] = s * dx; out[1] = s * dy; out[2] = s * dz;
    return 1;
}

/* The same pair law with the separation formed in binary64, rounded to binary32, and every
 * later step in binary32; the three components are returned widened to binary64 for an FP64
 * accumulation. */
int orc_pair_force_f32(double xi, double yi, double zi, double di, double xj, double yj, double zj,
                       double dj, double k, double gamma, double out[3])
{
    out[0] = 0.0; out[1] = 0.0; out[2] = 0.0;
    float dx = (float)(xi - xj), dy = (float)(yi - yj), dz = (float)(zi - zj);
    float dist = sqrtf((dx * dx + dy * dy) + dz * dz);
    float ri = (float)(0.5 * di), rj = (float)(0.5 * dj);
    float delta = (ri + rj) - dist;
    if (!(delta > 0.0f)) return 0;
    if (dist == 0.0f) return 1;
    float rhat = (ri * rj) / (ri + rj);
    float F = (float)k * delta - (float)gamma * sqrtf(rhat * delta);
    float s = F / dist;
    out[0] = (double)(s * dx); out[1] = (double)(s * dy); out[2] = (double)(s * dz);
    return 1;
}

/* Displacement of one agent from its summed force: no movement when |F| < adh; otherwise
 * disp = dt * F, rescaled to length max_disp when longer than that.  Returns 1 when gated,
 * 2 when clamped, 0 otherwise. */
int orc_displacement(double fx, double fy, double fz, double adh, double dt, double max_disp,
                     double disp[3])
{
    disp[0] = 0.0; disp[1] = 0.0; disp[2] = 0.0;
    double fnorm = sqrt((fx * fx + fy * fy) + fz * fz);
    if (fnorm < adh) return 1;
    double ux = dt * fx, uy = dt * fy, uz = dt * fz;
    double len = sqrt((ux * ux + uy * uy) + uz * uz);
    int clamped = 0;
    if (len > max_disp) {
        double scale = max_disp / len;
        ux = ux * scale; uy = uy * scale; uz = uz * scale;
        clamped = 2;
    }
    disp[0] = ux; disp[1] = uy; disp[2] = uz;
    return clamped;
}

typedef struct {
    double k, gamma, dt, max_disp, box;
    int32_t force_bits;   /* 64 or 32 */
    int64_t max_boxes;
} orc_mech_params;

/* Summed force on agent i: the 27 boxes around its own are visited in ascending key order and
 * the agents of each box in ascending id, skipping i itself.  Returns the contact count. */
static uint32_t agent_force(int64_t i, const double *x, const double *y, const double *z,
                            const double *d, const orc_mech_params *p, const orc_grid *g,
                            const uint32_t *order, const uint32_t *start, double f_out[3])
{
    int64_t cx = box_coord(g, x[i], 0), cy = box_coord(g, y[i], 1), cz = box_coord(g, z[i], 2);
    double sx = 0.0, sy = 0.0, sz = 0.0;
    uint32_t contacts = 0;
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                int64_t nk = neighbour_key(g, cx, cy, cz, ox, oy, oz);
                if (nk < 0) continue;
                for (uint32_t s = start[nk]; s < start[nk + 1]; ++s) {
                    uint32_t j = order[s];
                    if ((int64_t)j == i) continue;
                    double f[3];
                    int hit = (p->force_bits == 32)
                                  ? orc_pair_force_f32(x[i], y[i], z[i], d[i], x[j], y[j], z[j], d[j],
                                                       p->k, p->gamma, f)
                                  : orc_pair_force_f64(x[i], y[i], z[i], d[i], x[j], y[j], z[j], d[j],
                                                       p->k, p->gamma, f);
                    if (hit) {
                        contacts += 1;
                        sx = sx + f[0]; sy = sy + f[1]; sz = sz + f[2];
                    }
                }
            }
    f_out[0] = sx; f_out[1] = sy; f_out[2] = sz;
    return contacts;
}

/* Summed force on every agent.  ncontact (optional) receives each agent's contact count. */
static int mech_forces(int64_t n, const double *x, const double *y, const double *z,
                       const double *d, const orc_mech_params *p, const orc_grid *g,
                       const uint32_t *order, const uint32_t *start,
                       double *fx, double *fy, double *fz, uint32_t *ncontact)
{
    for (int64_t i = 0; i < n; ++i) {
        double f[3];
        uint32_t c = agent_force(i, x, y, z, d, p, g, order, start, f);
        fx[i] = f[0]; fy[i] = f[1]; fz[i] = f[2];
        if (ncontact) ncontact[i] = c;
    }
    return ORC_OK;
}

static int check_mech_params(const orc_mech_params *p)
{
    if (!(p->dt > 0.0) || !(p->max_disp > 0.0) || !isfinite(p->k) || !isfinite(p->gamma))
        return ORC_EINVAL;
    if (p->force_bits != 64 && p->force_bits != 32) return ORC_EINVAL;
    return ORC_OK;
}

/* One mechanical step (open space): grid on positions at t, summed forces, then every position
 * moved synchronously.  fx/fy/fz receive the summed (pre-gate) forces.  Optional outputs:
 * ncontact[n]; flags[n] (1 gated, 2 clamped, 0 moved freely). */
int orc_mech_step(int64_t n, double *x, double *y, double *z, const double *d, const double *adh,
                  const orc_mech_params *p, double *fx, double *fy, double *fz, uint32_t *ncontact,
                  uint8_t *flags)
{
    int rc = check_mech_params(p);
    if (rc) return rc;
    if (n == 0) return ORC_OK;
    orc_grid g;
    rc = orc_grid_setup(n, x, y, z, d, p->box, 0, 0.0, p->max_boxes, &g);
    if (rc) return rc;
    uint32_t *key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *start = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g.nboxes + 1));
    if (!key || !order || !start) { free(key); free(order); free(start); return ORC_ENOMEM; }
    rc = orc_grid_sort(n, x, y, z, &g, key, order, start);
    if (!rc) rc = mech_forces(n, x, y, z, d, p, &g, order, start, fx, fy, fz, ncontact);
    if (!rc) {
        for (int64_t i = 0; i < n; ++i) {
            double disp[3];
            int f = orc_displacement(fx[i], fy[i], fz[i], adh[i], p->dt, p->max_disp, disp);
            if (flags) flags[i] = (uint8_t)f;
            if (f == 1) continue; /* gated: the position stays bit-identical */
            x[i] = x[i] + disp[0];
            y[i] = y[i] + disp[1];
            z[i] = z[i] + disp[2];
        }
    }
    free(key); free(order); free(start);
    return rc;
}

/* The summed (pre-gate) forces of the m agents ids[0..m) of one mechanical step on positions
 * at t, each exactly as orc_mech_step computes it (same grid, same candidate order): for
 * checking sampled agents of populations too large to step whole on one core. */
int orc_mech_sample(int64_t n, const double *x, const double *y, const double *z, const double *d,
                    const orc_mech_params *p, int64_t m, const int64_t *ids, double *fx, double *fy,
                    double *fz, uint32_t *ncontact)
{
    int rc = check_mech_params(p);
    if (rc) return rc;
    if (n == 0 || m == 0) return ORC_OK;
    for (int64_t k = 0; k < m; ++k)
        if (ids[k] < 0 || ids[k] >= n) return ORC_EINVAL;
    orc_grid g;
    rc = orc_grid_setup(n, x, y, z, d, p->box, 0, 0.0, p->max_boxes, &g);
    if (rc) return rc;
    uint32_t *key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *start = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g.nboxes + 1));
    if (!key || !order || !start) { free(key); free(order); free(start); return ORC_ENOMEM; }
    rc = orc_grid_sort(n, x, y, z, &g, key, order, start);
    for (int64_t k = 0; !rc && k < m; ++k) {
        double f[3];
        uint32_t c = agent_force(ids[k], x, y, z, d, p, &g, order, start, f);
        fx[k] = f[0]; fy[k] = f[1]; fz[k] = f[2];
        if (ncontact) ncontact[k] = c;
    }
    free(key); free(order); free(start);
    return rc;
}

/* Contact lists in canonical order (the candidate order of the force sum).  First call with
 * ids == NULL to get counts[n]; then with ids sized sum(counts) and offsets[n] (exclusive prefix
 * of counts) to receive the contact ids of each agent.  periodic selects the SIR notion
 * (min-image squared distance <= radius^2); otherwise the mechanical contact delta > 0 of the
 * force_bits law. */
int orc_contacts(int64_t n, const double *x, const double *y, const double *z, const double *d,
                 double box, int32_t periodic, double L, double radius, int32_t force_bits,
                 int64_t max_boxes, uint32_t *counts, const int64_t *offsets, uint32_t *ids)
{
    orc_grid g;
    if (n == 0) return ORC_OK;
    int rc = orc_grid_setup(n, x, y, z, d, box, periodic, L, max_boxes, &g);
    if (rc) return rc;
    uint32_t *key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *start = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g.nboxes + 1));
    if (!key || !order || !start) { free(key); free(order); free(start); return ORC_ENOMEM; }
    rc = orc_grid_sort(n, x, y, z, &g, key, order, start);
    double r2 = radius * radius, half = 0.5 * L;
    for (int64_t i = 0; i < n && !rc; ++i) {
        int64_t cx = box_coord(&g, x[i], 0), cy = box_coord(&g, y[i], 1), cz = box_coord(&g, z[i], 2);
        uint32_t cnt = 0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int64_t nk = neighbour_key(&g, cx, cy, cz, ox, oy, oz);
                    if (nk < 0) continue;
                    for (uint32_t s = start[nk]; s < start[nk + 1]; ++s) {
                        uint32_t j = order[s];
                        if ((int64_t)j == i) continue;
                        int hit;
                        if (periodic) {
                            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
                            if (dx > half) dx -= L; else if (dx < -half) dx += L;
                            if (dy > half) dy -= L; else if (dy < -half) dy += L;
                            if (dz > half) dz -= L; else if (dz < -half) dz += L;
                            hit = ((dx * dx + dy * dy) + dz * dz) <= r2;
                        } else {
                            double f[3];
                            hit = (force_bits == 32)
                                      ? orc_pair_force_f32(x[i], y[i], z[i], d[i], x[j], y[j], z[j],
                                                           d[j], 1.0, 0.0, f)
                                      : orc_pair_force_f64(x[i], y[i], z[i], d[i], x[j], y[j], z[j],
                                                           d[j], 1.0, 0.0, f);
                        }
                        if (hit) {
                            if (ids) ids[offsets[i] + cnt] = j;
                            cnt += 1;
                        }
                    }
                }
        counts[i] = cnt;
    }
    free(key); free(order); free(start);
    return rc;
}

/* ------------------------------------------------------------------------------------------ */
/* Tumour spheroid: growth and division [Sec. 3.2], then the mechanical step                   */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    orc_mech_params mech;
    double grow;       /* diameter factor per step (cube root of the volume factor) */
    double div_d;      /* division threshold diameter */
    double half_cbrt;  /* daughter diameter factor, cube root of 1/2 */
    uint64_t seed, salt;
} orc_spheroid_params;

/* Division axis of mother `id` at `step`: rejection from [-1, 1)^3 with attempt counter,
 * accepting 0 < |v|^2 <= 1, normalised by sqrt(|v|^2); (1, 0, 0) after 64 rejections. */
void orc_division_axis(uint64_t seed, uint64_t salt, uint64_t id, uint64_t step, double u[3])
{
    u[0] = 1.0; u[1] = 0.0; u[2] = 0.0;
    for (uint64_t attempt = 0; attempt < 64; ++attempt) {
        uint64_t w[4];
        orc_draw(seed, salt, RNG_DIV, attempt, id, step, w);
        double vx = 2.0 * orc_u01(w[0]) - 1.0;
        double vy = 2.0 * orc_u01(w[1]) - 1.0;
        double vz = 2.0 * orc_u01(w[2]) - 1.0;
        double s = (vx * vx + vy * vy) + vz * vz;
        if (s > 0.0 && s <= 1.0) {
            double norm = sqrt(s);
            u[0] = vx / norm; u[1] = vy / norm; u[2] = vz / norm;
            return;
        }
    }
}

/* Growth and division of one step.  Every diameter is multiplied by `grow`; then each agent
 * with d >= div_d, taken in ascending id, divides: d' = d * half_cbrt, the mother moves to
 * x - (d'/4)*u and the daughter appears at x + (d'/4)*u along the random axis u, with the same
 * adherence.  The daughter of the r-th dividing mother (by id) gets id n + r.  Divisions whose
 * daughter id would reach `capacity` do not happen (the mother keeps growing) and *overflow is
 * set.  *n is updated. */
int orc_grow_divide(int64_t *n, int64_t capacity, double *x, double *y, double *z, double *d,
                    double *adh, const orc_spheroid_params *p, int64_t step, int32_t *overflow)
{
    int64_t n0 = *n, next = n0;
    if (overflow) *overflow = 0;
    for (int64_t i = 0; i < n0; ++i) d[i] = d[i] * p->grow;
    for (int64_t i = 0; i < n0; ++i) {
        if (!(d[i] >= p->div_d)) continue;
        if (next >= capacity) {
            if (overflow) *overflow = 1;
            continue;
        }
        double u[3];
        orc_division_axis(p->seed, p->salt, (uint64_t)i, (uint64_t)step, u);
        double dp = d[i] * p->half_cbrt;
        double q = 0.25 * dp;
        double ox = q * u[0], oy = q * u[1], oz = q * u[2];
        int64_t j = next++;
        x[j] = x[i] + ox; y[j] = y[i] + oy; z[j] = z[i] + oz;
        d[j] = dp; adh[j] = adh[i];
        x[i] = x[i] - ox; y[i] = y[i] - oy; z[i] = z[i] - oz;
        d[i] = dp;
    }
    *n = next;
    return ORC_OK;
}

/* One spheroid step: grow -> divide -> grid -> mechanics. */
int orc_spheroid_step(int64_t *n, int64_t capacity, double *x, double *y, double *z, double *d,
                      double *adh, const orc_spheroid_params *p, int64_t step, double *fx,
                      double *fy, double *fz, int32_t *overflow)
{
    int rc = check_mech_params(&p->mech);
    if (rc) return rc;
    rc = orc_grow_divide(n, capacity, x, y, z, d, adh, p, step, overflow);
    if (rc) return rc;
    return orc_mech_step(*n, x, y, z, d, adh, &p->mech, fx, fy, fz, NULL, NULL);
}

/* ------------------------------------------------------------------------------------------ */
/* Tumour spheroid with apoptosis and Brownian migration [Sec. 3.2]                            */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    orc_spheroid_params sph;  /* growth, division, mechanics, Philox key */
    double p_apo;             /* probability per step that a cell dies */
    double migrate;           /* bound of the Brownian displacement per axis and step */
} orc_oncology_params;

/* Apoptosis.  Cell `id` dies at `step` iff word 0 of the draw (APO, 0, id, step) is below
 * floor(p_apo * 2^64).  The survivors keep their relative order by id and are renumbered
 * 0 .. n'-1 in that order, so ids stay dense (the next daughter id is n').  *n is updated. */
int orc_apoptosis(int64_t *n, double *x, double *y, double *z, double *d, double *adh,
                  double p_apo, uint64_t seed, uint64_t salt, int64_t step)
{
    int64_t n0 = *n, kept = 0;
    for (int64_t i = 0; i < n0; ++i) {
        uint64_t w[4];
        orc_draw(seed, salt, RNG_APO, 0, (uint64_t)i, (uint64_t)step, w);
        if (orc_bernoulli(w[0], p_apo)) continue;
        x[kept] = x[i]; y[kept] = y[i]; z[kept] = z[i];
        d[kept] = d[i]; adh[kept] = adh[i];
        ++kept;
    }
    *n = kept;
    return ORC_OK;
}

/* Brownian migration: every cell moves by migrate * (2u - 1) per axis, with u from words 0..2
 * of the draw (MIG, 0, id, step).  Open space: no wall, no wrap. */
int orc_migrate(int64_t n, double *x, double *y, double *z, double migrate, uint64_t seed,
                uint64_t salt, int64_t step)
{
    if (!(migrate >= 0.0) || !isfinite(migrate)) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t w[4];
        orc_draw(seed, salt, RNG_MIG, 0, (uint64_t)i, (uint64_t)step, w);
        x[i] = x[i] + migrate * (2.0 * orc_u01(w[0]) - 1.0);
        y[i] = y[i] + migrate * (2.0 * orc_u01(w[1]) - 1.0);
        z[i] = z[i] + migrate * (2.0 * orc_u01(w[2]) - 1.0);
    }
    return ORC_OK;
}

/* One step of the tumour-spheroid behaviour: apoptosis -> growth -> division -> migration ->
 * grid -> mechanics.  Each part draws with the ids the cells hold when it runs (the division
 * axis and the migration use the ids after the renumbering of this step's apoptosis; a daughter
 * migrates with its own new id). */
int orc_oncology_step(int64_t *n, int64_t capacity, double *x, double *y, double *z, double *d,
                      double *adh, const orc_oncology_params *p, int64_t step, double *fx,
                      double *fy, double *fz, int32_t *overflow)
{
    int rc = check_mech_params(&p->sph.mech);
    if (rc) return rc;
    if (!(p->p_apo >= 0.0) || !(p->p_apo <= 1.0) || !(p->migrate >= 0.0) || !isfinite(p->migrate))
        return ORC_EINVAL;
    rc = orc_apoptosis(n, x, y, z, d, adh, p->p_apo, p->sph.seed, p->sph.salt, step);
    if (rc) return rc;
    rc = orc_grow_divide(n, capacity, x, y, z, d, adh, &p->sph, step, overflow);
    if (rc) return rc;
    rc = orc_migrate(*n, x, y, z, p->migrate, p->sph.seed, p->sph.salt, step);
    if (rc) return rc;
    return orc_mech_step(*n, x, y, z, d, adh, &p->sph.mech, fx, fy, fz, NULL, NULL);
}

/* ------------------------------------------------------------------------------------------ */
/* SIR epidemiology [Sec. 3.3]                                                                 */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    double L;        /* periodic cube edge */
    double box;      /* requested box edge (>= infection radius) */
    double r_inf;    /* infection radius (inclusive) */
    double p_inf;    /* infection probability per infected contact and step */
    double p_rec;    /* recovery probability per step */
    double walk;     /* maximum displacement per axis and step */
    int64_t max_boxes;
    uint64_t seed, salt;
} orc_sir_params;

enum { SIR_S = 0, SIR_I = 1, SIR_R = 2 };

/* One SIR step.  Everything reads the state and positions at t and writes t+1:
 *  - a susceptible agent counts m infected agents within the infection radius (periodic
 *    minimum image, squared distance <= r_inf^2) and becomes infected iff one of the m
 *    independent per-contact draws (INF, attempt c, id, t), c < m, succeeds with p_inf;
 *  - an infected agent recovers iff its draw (REC, 0, id, t) succeeds with p_rec;
 *  - every agent moves by walk*(2u - 1) per axis with u from words 0..2 of (MOVE, 0, id, t),
 *    then wraps into [0, L): below 0 add L, at or above L subtract L, a result equal to L is 0.
 * counts[3] receives the S, I, R totals at t+1. */
int orc_sir_step(int64_t n, double *x, double *y, double *z, uint8_t *state,
                 const orc_sir_params *p, int64_t step, int64_t counts[3])
{
    if (!(p->r_inf >= 0.0) || p->box < p->r_inf || !(p->walk >= 0.0) || p->walk > p->L)
        return ORC_EINVAL;
    counts[0] = counts[1] = counts[2] = 0;
    if (n == 0) return ORC_OK;
    orc_grid g;
    int rc = orc_grid_setup(n, x, y, z, NULL, p->box, 1, p->L, p->max_boxes, &g);
    if (rc) return rc;
    uint32_t *key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *start = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g.nboxes + 1));
    uint8_t *next = (uint8_t *)malloc((size_t)n);
    if (!key || !order || !start || !next) {
        free(key); free(order); free(start); free(next);
        return ORC_ENOMEM;
    }
    rc = orc_grid_sort(n, x, y, z, &g, key, order, start);
    double r2 = p->r_inf * p->r_inf, half = 0.5 * p->L;
    for (int64_t i = 0; i < n && !rc; ++i) {
        uint8_t s = state[i];
        if (s == SIR_S) {
            int64_t cx = box_coord(&g, x[i], 0), cy = box_coord(&g, y[i], 1);
            int64_t cz = box_coord(&g, z[i], 2);
            uint64_t m = 0;
            for (int oz = -1; oz <= 1; ++oz)
                for (int oy = -1; oy <= 1; ++oy)
                    for (int ox = -1; ox <= 1; ++ox) {
                        int64_t nk = neighbour_key(&g, cx, cy, cz, ox, oy, oz);
                        for (uint32_t q = start[nk]; q < start[nk + 1]; ++q) {
                            uint32_t j = order[q];
                            if ((int64_t)j == i || state[j] != SIR_I) continue;
                            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
                            if (dx > half) dx -= p->L; else if (dx < -half) dx += p->L;
                            if (dy > half) dy -= p->L; else if (dy < -half) dy += p->L;
                            if (dz > half) dz -= p->L; else if (dz < -half) dz += p->L;
                            if ((dx * dx + dy * dy) + dz * dz <= r2) m += 1;
                        }
                    }
            uint8_t ns = SIR_S;
            for (uint64_t c = 0; c < m; ++c) {
                uint64_t w[4];
                orc_draw(p->seed, p->salt, RNG_INF, c, (uint64_t)i, (uint64_t)step, w);
                if (orc_bernoulli(w[0], p->p_inf)) { ns = SIR_I; break; }
            }
            next[i] = ns;
        } else if (s == SIR_I) {
            uint64_t w[4];
            orc_draw(p->seed, p->salt, RNG_REC, 0, (uint64_t)i, (uint64_t)step, w);
            next[i] = orc_bernoulli(w[0], p->p_rec) ? SIR_R : SIR_I;
        } else {
            next[i] = SIR_R;
        }
    }
    if (!rc) {
        for (int64_t i = 0; i < n; ++i) {
            uint64_t w[4];
            orc_draw(p->seed, p->salt, RNG_MOVE, 0, (uint64_t)i, (uint64_t)step, w);
            double *pos[3] = {&x[i], &y[i], &z[i]};
            for (int a = 0; a < 3; ++a) {
                double v = *pos[a] + p->walk * (2.0 * orc_u01(w[a]) - 1.0);
                if (v < 0.0) v += p->L;
                if (v >= p->L) v -= p->L;
                if (v == p->L) v = 0.0;
                *pos[a] = v;
            }
            state[i] = next[i];
            counts[next[i]] += 1;
        }
    }
    free(key); free(order); free(start); free(next);
    return rc;
}

/* ------------------------------------------------------------------------------------------ */
/* Extracellular substances [Sec. 2.1: diffusion of substances as a standalone operation run   */
/* once per step; secretion and chemotaxis as agent behaviours] and the soma-clustering        */
/* benchmark [Sec. 3.4]                                                                        */
/* ------------------------------------------------------------------------------------------ */
/* A substance lives on a uniform grid of nx*ny*nz cubic voxels of edge h with lower corner
 * (x0, y0, z0); voxel (i, j, k) is element i + nx*(j + ny*k) (x fastest).  The two substances of
 * the soma-clustering model are stored one after the other (substance s at offset s*V). */
typedef struct {
    int64_t nx, ny, nz;
    double x0, y0, z0, h;
} orc_field;

static int check_field(const orc_field *f)
{
    if (f->nx < 1 || f->ny < 1 || f->nz < 1) return ORC_EINVAL;
    if (!(f->h > 0.0) || !isfinite(f->h) || !finite3(f->x0, f->y0, f->z0)) return ORC_EINVAL;
    return ORC_OK;
}

static int64_t field_index(const orc_field *f, int64_t i, int64_t j, int64_t k)
{
    return i + f->nx * (j + f->ny * k);
}

/* Voxel coordinate of a position along one axis: floor((v - origin) / h), clamped into the grid
 * (agents outside the grid use the nearest boundary voxel). */
static int64_t voxel_coord(double v, double origin, double h, int64_t n)
{
    double c = floor((v - origin) / h);
    if (c < 0.0) c = 0.0;
    if (c > (double)(n - 1)) c = (double)(n - 1);
    return (int64_t)c;
}

/* One explicit (forward-Euler, central-difference) diffusion step with decay:
 *   out = c + (lam * L(c) - kdec * c),
 *   L(c) = ((dx- + dx+) + (dy- + dy+)) + (dz- + dz+),  d = c_neighbour - c,
 * lam = D*dt/h^2 and kdec = decay*dt.  The boundary is closed (no flux): a neighbour outside the
 * grid takes the voxel's own value, so its difference is zero. */
int orc_diffuse(const orc_field *f, const double *in, double *out, double lam, double kdec)
{
    int rc = check_field(f);
    if (rc) return rc;
    for (int64_t k = 0; k < f->nz; ++k)
        for (int64_t j = 0; j < f->ny; ++j)
            for (int64_t i = 0; i < f->nx; ++i) {
                double c = in[field_index(f, i, j, k)];
                double xm = i > 0 ? in[field_index(f, i - 1, j, k)] : c;
                double xp = i < f->nx - 1 ? in[field_index(f, i + 1, j, k)] : c;
                double ym = j > 0 ? in[field_index(f, i, j - 1, k)] : c;
                double yp = j < f->ny - 1 ? in[field_index(f, i, j + 1, k)] : c;
                double zm = k > 0 ? in[field_index(f, i, j, k - 1)] : c;
                double zp = k < f->nz - 1 ? in[field_index(f, i, j, k + 1)] : c;
                double lap = (((xm - c) + (xp - c)) + ((ym - c) + (yp - c))) + ((zm - c) + (zp - c));
                out[field_index(f, i, j, k)] = c + (lam * lap - kdec * c);
            }
    return ORC_OK;
}

/* Coefficients of the diffusion step from the physical parameters (the same expressions on
 * every side): lam = (D*dt)/(h*h), kdec = decay*dt. */
void orc_diffusion_coefficients(double D, double decay, double dt, double h, double out[2])
{
    out[0] = (D * dt) / (h * h);
    out[1] = decay * dt;
}

/* Secretion: every agent of type s (0 or 1) adds q to substance s in the voxel holding its
 * centre; a voxel holding m such agents gains q*m at once: c = c + q*m.  Agents of any other
 * type are inert. */
int orc_secrete(const orc_field *f, int64_t n, const double *x, const double *y, const double *z,
                const uint8_t *type, double q, double *c)
{
    int rc = check_field(f);
    if (rc) return rc;
    int64_t V = f->nx * f->ny * f->nz;
    uint32_t *m = (uint32_t *)calloc((size_t)(2 * V), sizeof(uint32_t));
    if (!m) return ORC_ENOMEM;
    for (int64_t a = 0; a < n; ++a) {
        if (type[a] > 1) continue;
        int64_t v = field_index(f, voxel_coord(x[a], f->x0, f->h, f->nx),
                                voxel_coord(y[a], f->y0, f->h, f->ny),
                                voxel_coord(z[a], f->z0, f->h, f->nz));
        m[type[a] * V + v] += 1;
    }
    for (int64_t v = 0; v < 2 * V; ++v)
        if (m[v]) c[v] = c[v] + q * (double)m[v];
    free(m);
    return ORC_OK;
}

/* Chemotaxis: an agent of type s moves by `speed` along the gradient of substance s at its
 * voxel, g = (c(i+1) - c(i-1), c(j+1) - c(j-1), c(k+1) - c(k-1)) with neighbours outside the grid
 * taking the voxel's own value; x += (speed/|g|) * g with |g| = sqrt((gx*gx + gy*gy) + gz*gz);
 * no move where g = 0.  Agents of any other type do not move. */
int orc_chemotaxis(const orc_field *f, int64_t n, double *x, double *y, double *z,
                   const uint8_t *type, const double *c, double speed)
{
    int rc = check_field(f);
    if (rc) return rc;
    int64_t V = f->nx * f->ny * f->nz;
    for (int64_t a = 0; a < n; ++a) {
        if (type[a] > 1) continue;
        const double *cs = c + type[a] * V;
        int64_t i = voxel_coord(x[a], f->x0, f->h, f->nx);
        int64_t j = voxel_coord(y[a], f->y0, f->h, f->ny);
        int64_t k = voxel_coord(z[a], f->z0, f->h, f->nz);
        int64_t im = i > 0 ? i - 1 : i, ip = i < f->nx - 1 ? i + 1 : i;
        int64_t jm = j > 0 ? j - 1 : j, jp = j < f->ny - 1 ? j + 1 : j;
        int64_t km = k > 0 ? k - 1 : k, kp = k < f->nz - 1 ? k + 1 : k;
        double gx = cs[field_index(f, ip, j, k)] - cs[field_index(f, im, j, k)];
        double gy = cs[field_index(f, i, jp, k)] - cs[field_index(f, i, jm, k)];
        double gz = cs[field_index(f, i, j, kp)] - cs[field_index(f, i, j, km)];
        double g2 = (gx * gx + gy * gy) + gz * gz;
        if (!(g2 > 0.0)) continue;
        double s = speed / sqrt(g2);
        x[a] = x[a] + s * gx;
        y[a] = y[a] + s * gy;
        z[a] = z[a] + s * gz;
    }
    return ORC_OK;
}

typedef struct {
    orc_mech_params mech;  /* mechanics; mech.dt is also the diffusion time step */
    double D;              /* diffusion coefficient */
    double decay;          /* decay rate */
    double secrete;        /* quantity an agent adds to its substance per step */
    double speed;          /* chemotactic displacement per step */
} orc_soma_params;

/* One soma-clustering step: secretion into c (in place) -> one diffusion step of both substances
 * c -> c_next -> chemotaxis on c_next -> grid -> mechanics.  type[] is the agent's cell type. */
int orc_soma_step(int64_t n, double *x, double *y, double *z, const double *d, const double *adh,
                  const uint8_t *type, const orc_field *f, double *c, double *c_next,
                  const orc_soma_params *p, double *fx, double *fy, double *fz)
{
    int rc = check_mech_params(&p->mech);
    if (rc) return rc;
    rc = check_field(f);
    if (rc) return rc;
    double coef[2];
    orc_diffusion_coefficients(p->D, p->decay, p->mech.dt, f->h, coef);
    if (!(coef[0] >= 0.0) || coef[0] > 1.0 / 6.0 || !(coef[1] >= 0.0) || coef[1] > 1.0) return ORC_EINVAL;
    if (!isfinite(p->secrete) || !(p->speed >= 0.0) || !isfinite(p->speed)) return ORC_EINVAL;
    rc = orc_secrete(f, n, x, y, z, type, p->secrete, c);
    if (rc) return rc;
    int64_t V = f->nx * f->ny * f->nz;
    for (int s = 0; s < 2 && !rc; ++s) rc = orc_diffuse(f, c + s * V, c_next + s * V, coef[0], coef[1]);
    if (rc) return rc;
    rc = orc_chemotaxis(f, n, x, y, z, type, c_next, p->speed);
    if (rc) return rc;
    return orc_mech_step(n, x, y, z, d, adh, &p->mech, fx, fy, fz, NULL, NULL);
}

/* ------------------------------------------------------------------------------------------ */
/* Cylinder geometry: neurite elements [Sec. 2.2, neuroscience module]                        */
/* ------------------------------------------------------------------------------------------ */
/* A neurite element is a cylinder from its proximal end p to its distal end q, where its point
 * mass sits; its agent position is q.  Spheres and cylinders share the grid: an agent's grid
 * diameter is the diameter of the smallest sphere about its position that holds its whole
 * geometry (a sphere's own diameter; 2|q - p| + dc for a cylinder of diameter dc), so the box
 * edge (the largest grid diameter) still finds every contact in the 27 boxes.
 *
 * Contact geometry: the closest points of the two bodies' axes (a sphere's axis is its centre)
 * carry virtual spheres of the bodies' diameters, and the sphere-sphere law acts between them.
 * A cylinder's point mass takes the share t of the force, t in [0, 1] being the position of its
 * closest point along p -> q (1 at the distal end); the remainder would act on its proximal end,
 * which belongs to the element it grows from and does not move in this step. */
enum { GEOM_SPHERE = 0, GEOM_CYLINDER = 1 };

static double dot3(const double a[3], const double b[3]) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* Parameter t in [0, 1] of the point of segment p -> q closest to c: t = ((c - p).d)/(d.d),
 * d = q - p, clamped.  A segment of length 0 is its distal point: t = 1. */
double orc_segment_point_param(const double p[3], const double q[3], const double c[3])
{
    double d[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    double w[3] = {c[0] - p[0], c[1] - p[1], c[2] - p[2]};
    double a = dot3(d, d);
    if (!(a > 0.0)) return 1.0;
    return clamp01(dot3(w, d) / a);
}

/* Parameters (s, t) of the closest points of segments p1 -> q1 and p2 -> q2, from minimising
 * |p1 + s d1 - p2 - t d2|^2 over [0, 1]^2: with r = p1 - p2, a = d1.d1, e = d2.d2, b = d1.d2,
 * c = d1.r, f = d2.r, the unconstrained s = (b f - c e)/(a e - b^2) is clamped, t = (b s + f)/e
 * follows, and when t leaves [0, 1] it is clamped and s recomputed for that t.  Segments within
 * an angle of about 1e-6 rad of parallel (a e - b^2 <= 2^-40 a e) start from s = 0.  A segment
 * of length 0 is its distal point (parameter 1). */
void orc_segment_segment_params(const double p1[3], const double q1[3], const double p2[3],
                                const double q2[3], double *s_out, double *t_out)
{
    double d1[3] = {q1[0] - p1[0], q1[1] - p1[1], q1[2] - p1[2]};
    double d2[3] = {q2[0] - p2[0], q2[1] - p2[1], q2[2] - p2[2]};
    double r[3] = {p1[0] - p2[0], p1[1] - p2[1], p1[2] - p2[2]};
    double a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r);
    double s = 0.0, t = 0.0;
    if (!(a > 0.0) && !(e > 0.0)) {
        s = 1.0; t = 1.0;
    } else if (!(a > 0.0)) {
        s = 1.0; t = clamp01(f / e);
    } else {
        double c = dot3(d1, r);
        if (!(e > 0.0)) {
            t = 1.0; s = clamp01(-c / a);
        } else {
            double b = dot3(d1, d2);
            double ae = a * e;
            double denom = ae - b * b;
            s = denom > 0x1.0p-40 * ae ? clamp01((b * f - c * e) / denom) : 0.0;
            double tn = b * s + f;
            if (tn < 0.0) {
                t = 0.0; s = clamp01(-c / a);
            } else if (tn > e) {
                t = 1.0; s = clamp01((b - c) / a);
            } else {
                t = tn / e;
            }
        }
    }
    *s_out = s; *t_out = t;
}

/* Grid diameter of a cylinder from p to q of diameter dc: 2|q - p| + dc. */
double orc_cylinder_reach(const double p[3], const double q[3], double dc)
{
    double d[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    return 2.0 * sqrt(dot3(d, d)) + dc;
}

/* Force on body i from body j.  Body = (kind, position x = centre or distal end, diameter d of a
 * sphere, proximal end p and diameter dc of a cylinder).  Returns 1 on contact and writes the
 * force on i (for a cylinder: the share that acts on its point mass). */
int orc_geom_pair(int kind_i, const double xi[3], double di, const double pi_[3], double dci,
                  int kind_j, const double xj[3], double dj, const double pj[3], double dcj,
                  double k, double gamma, double out[3])
{
    double ci[3], cj[3], Di, Dj, share = 1.0;
    if (kind_i == GEOM_CYLINDER && kind_j == GEOM_CYLINDER) {
        double s, t;
        orc_segment_segment_params(pi_, xi, pj, xj, &s, &t);
        for (int a = 0; a < 3; ++a) {
            ci[a] = pi_[a] + s * (xi[a] - pi_[a]);
            cj[a] = pj[a] + t * (xj[a] - pj[a]);
        }
        Di = dci; Dj = dcj; share = s;
    } else if (kind_i == GEOM_CYLINDER) {
        double s = orc_segment_point_param(pi_, xi, xj);
        for (int a = 0; a < 3; ++a) {
            ci[a] = pi_[a] + s * (xi[a] - pi_[a]);
            cj[a] = xj[a];
        }
        Di = dci; Dj = dj; share = s;
    } else if (kind_j == GEOM_CYLINDER) {
        double t = orc_segment_point_param(pj, xj, xi);
        for (int a = 0; a < 3; ++a) {
            ci[a] = xi[a];
            cj[a] = pj[a] + t * (xj[a] - pj[a]);
        }
        Di = di; Dj = dcj;
    } else {
        for (int a = 0; a < 3; ++a) { ci[a] = xi[a]; cj[a] = xj[a]; }
        Di = di; Dj = dj;
    }
    int hit = orc_pair_force_f64(ci[0], ci[1], ci[2], Di, cj[0], cj[1], cj[2], Dj, k, gamma, out);
    out[0] = share * out[0]; out[1] = share * out[1]; out[2] = share * out[2];
    return hit;
}

/* One mechanical step of spheres and cylinders (binary64 law).  kind[i] = 1 marks a cylinder
 * whose proximal end and diameter are (px, py, pz)[i], dc[i]; every other kind is a sphere of
 * diameter d[i].  First each cylinder's d[i] is set to its grid diameter (orc_cylinder_reach),
 * then the grid is built.  Forces are summed in ascending (key, id) candidate order from +0.0;
 * the gate, the clamp and the synchronous update are those of the sphere step; a cylinder moves
 * its distal end only.  fx/fy/fz receive the summed forces (on a cylinder's point mass);
 * ncontact (optional) each agent's contact count. */
int orc_geom_step(int64_t n, double *x, double *y, double *z, double *d, const double *adh,
                  const uint8_t *kind, const double *px, const double *py, const double *pz,
                  const double *dc, const orc_mech_params *p, double *fx, double *fy, double *fz,
                  uint32_t *ncontact)
{
    int rc = check_mech_params(p);
    if (rc) return rc;
    if (p->force_bits != 64) return ORC_EINVAL;
    if (n == 0) return ORC_OK;
    for (int64_t i = 0; i < n; ++i) {
        if (kind[i] != GEOM_CYLINDER) continue;
        double q[3] = {x[i], y[i], z[i]}, pp[3] = {px[i], py[i], pz[i]};
        d[i] = orc_cylinder_reach(pp, q, dc[i]);
    }
    orc_grid g;
    rc = orc_grid_setup(n, x, y, z, d, p->box, 0, 0.0, p->max_boxes, &g);
    if (rc) return rc;
    uint32_t *key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *start = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g.nboxes + 1));
    if (!key || !order || !start) { free(key); free(order); free(start); return ORC_ENOMEM; }
    rc = orc_grid_sort(n, x, y, z, &g, key, order, start);
    for (int64_t i = 0; i < n && !rc; ++i) {
        int ki = kind[i] == GEOM_CYLINDER ? GEOM_CYLINDER : GEOM_SPHERE;
        double xi[3] = {x[i], y[i], z[i]}, pi_[3] = {px[i], py[i], pz[i]};
        int64_t cx = box_coord(&g, x[i], 0), cy = box_coord(&g, y[i], 1), cz = box_coord(&g, z[i], 2);
        double sx = 0.0, sy = 0.0, sz = 0.0;
        uint32_t contacts = 0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int64_t nk = neighbour_key(&g, cx, cy, cz, ox, oy, oz);
                    if (nk < 0) continue;
                    for (uint32_t s = start[nk]; s < start[nk + 1]; ++s) {
                        uint32_t j = order[s];
                        if ((int64_t)j == i) continue;
                        int kj = kind[j] == GEOM_CYLINDER ? GEOM_CYLINDER : GEOM_SPHERE;
                        double xj[3] = {x[j], y[j], z[j]}, pj[3] = {px[j], py[j], pz[j]};
                        double f[3];
                        if (orc_geom_pair(ki, xi, d[i], pi_, dc[i], kj, xj, d[j], pj, dc[j], p->k,
                                          p->gamma, f)) {
                            contacts += 1;
                            sx = sx + f[0]; sy = sy + f[1]; sz = sz + f[2];
                        }
                    }
                }
        fx[i] = sx; fy[i] = sy; fz[i] = sz;
        if (ncontact) ncontact[i] = contacts;
    }
    if (!rc) {
        for (int64_t i = 0; i < n; ++i) {
            double disp[3];
            if (orc_displacement(fx[i], fy[i], fz[i], adh[i], p->dt, p->max_disp, disp) == 1) continue;
            x[i] = x[i] + disp[0];
            y[i] = y[i] + disp[1];
            z[i] = z[i] + disp[2];
        }
    }
    free(key); free(order); free(start);
    return rc;
}
