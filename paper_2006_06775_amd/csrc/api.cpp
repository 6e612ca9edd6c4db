// api.cpp -- the C ABI of libbdm.so (declared in include/bdm.h).
//
// Host side only: synchronous argument validation, workspace layout, kernel launches on the
// caller's stream, error codes.  No allocation, no stream creation, no exceptions across the ABI.
// A plain call is a batch of one slot whose record travels by value in the kernel arguments.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "kernels.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(BDM_EHIP, "%s: %s", what, hipGetErrorString(e));
    return BDM_OK;
}

inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

bool is_fin(double v) { return std::isfinite(v); }

int check_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(BDM_ENODEV, "no HIP device");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(BDM_ENODEV, "no HIP device properties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BDM_ENODEV, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    return BDM_OK;
}

int view(void *ptr, size_t bytes, int64_t capacity, int64_t max_boxes, int64_t slots, bdm::Ws *out) {
    if (!ptr) return fail(BDM_ENOWS, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0) return fail(BDM_ENOWS, "workspace pointer is not 256-byte aligned");
    bdm::WsLayout lay;
    if (!bdm::ws_layout(capacity, max_boxes, slots, &lay))
        return fail(BDM_ENOWS, "workspace capacity %lld / max_boxes %lld / slots %lld out of range",
                    (long long)capacity, (long long)max_boxes, (long long)slots);
    if (bytes < lay.total) return fail(BDM_ENOWS, "workspace has %zu bytes, needs %zu", bytes, lay.total);
    *out = bdm::ws_view(ptr, lay);
    return BDM_OK;
}

int get_ws(const bdm_workspace *ws, bdm::Ws *out) {
    if (!ws) return fail(BDM_ENOWS, "workspace is NULL");
    return view(ws->ptr, ws->bytes, ws->capacity, ws->max_boxes, 0, out);
}

int get_batch(const bdm_batch *b, bdm::Ws *out) {
    if (!b) return fail(BDM_ENOWS, "batch is NULL");
    if (b->slots < 1 || b->slots > BDM_MAX_SLOTS) return fail(BDM_EINVAL, "batch slots must be in [1, %d]", BDM_MAX_SLOTS);
    if (b->grid_cap != 0 && b->grid_cap != -1 && (b->grid_cap < 64 || b->grid_cap > 65536))
        return fail(BDM_EINVAL, "batch grid_cap must be 0, -1 or in [64, 65536]");
    return view(b->ptr, b->bytes, b->capacity, b->max_boxes, b->slots, out);
}

int check_soa(const bdm_soa *s, int64_t ws_capacity, bool need_sphere, bool need_state) {
    if (!s) return fail(BDM_EINVAL, "soa is NULL");
    if (!s->n || !s->x || !s->y || !s->z || !s->id) return fail(BDM_EINVAL, "soa needs n, x, y, z and id");
    if (s->capacity < 0) return fail(BDM_EINVAL, "negative capacity");
    if (s->capacity > ws_capacity)
        return fail(BDM_ENOWS, "soa capacity %lld exceeds the workspace capacity %lld", (long long)s->capacity,
                    (long long)ws_capacity);
    if (need_sphere && (!s->diam || !s->adh)) return fail(BDM_EINVAL, "soa needs diam and adh");
    if (need_state && !s->state) return fail(BDM_EINVAL, "soa needs state");
    return BDM_OK;
}

// The stationary skip carries each agent's last force, so the steps that use it need them.
int check_skip(const bdm_soa *s, const bdm_params *p) {
    if (p->skip_static == 1 && !p->periodic && (!s->fx || !s->fy || !s->fz))
        return fail(BDM_EINVAL, "skip_static needs the force arrays fx, fy, fz");
    return BDM_OK;
}

int check_mech_params(const bdm_params *p) {
    if (!p) return fail(BDM_EINVAL, "params is NULL");
    if (!(p->dt > 0.0) || !is_fin(p->dt)) return fail(BDM_EINVAL, "dt must be > 0");
    if (!(p->max_disp > 0.0) || !is_fin(p->max_disp)) return fail(BDM_EINVAL, "max_disp must be > 0");
    if (!is_fin(p->k) || !is_fin(p->gamma)) return fail(BDM_EINVAL, "k and gamma must be finite");
    if (p->force_bits != 64 && p->force_bits != 32) return fail(BDM_EINVAL, "force_bits must be 32 or 64");
    if (!is_fin(p->box)) return fail(BDM_EINVAL, "box must be finite");
    if (p->periodic) return fail(BDM_EINVAL, "the mechanical step runs in open space (periodic = 0)");
    if (p->skip_static != 0 && p->skip_static != 1) return fail(BDM_EINVAL, "skip_static must be 0 or 1");
    return BDM_OK;
}

int periodic_boxes(const bdm_params *p, int64_t max_boxes, int32_t *nb) {
    if (!(p->L > 0.0) || !is_fin(p->L)) return fail(BDM_EINVAL, "periodic L must be > 0");
    if (!(p->box > 0.0) || !is_fin(p->box)) return fail(BDM_EINVAL, "periodic grids need box > 0");
    double q = std::floor(p->L / p->box);
    if (q < 3.0) return fail(BDM_EINVAL, "periodic grid needs at least 3 boxes per axis");
    if (q > 2097151.0 || q * q * q > double(max_boxes))
        return fail(BDM_ENOWS, "periodic grid of %.0f^3 boxes exceeds max_boxes %lld", q, (long long)max_boxes);
    *nb = int32_t(q);
    return BDM_OK;
}

// Slot record of a plain call (or of one batch slot).
bdm::SlotDev slot_record(const bdm_params *p, int64_t agent_off, int64_t capacity, int64_t box_off,
                         int64_t max_boxes, int64_t steps, bool has_d) {
    bdm::SlotDev r{};
    r.agent_off = agent_off;
    r.capacity = capacity;
    r.box_off = box_off;
    r.max_boxes = max_boxes;
    r.steps_left = steps;
    r.k = p->k;
    r.gamma = p->gamma;
    r.dt = p->dt;
    r.max_disp = p->max_disp;
    r.box = p->box;
    r.L = p->L;
    r.kf = float(p->k);
    r.gf = float(p->gamma);
    r.force_bits = p->force_bits;
    r.periodic = p->periodic ? 1 : 0;
    r.nb = 0;
    r.has_d = has_d ? 1 : 0;
    r.skip = p->skip_static == 1 ? 1 : 0;
    return r;
}

bdm::Slots plain_slots(const bdm::Ws &w, const bdm::SlotDev &rec) {
    bdm::Slots sl{};
    sl.table = nullptr;
    sl.tilemap = nullptr;
    sl.bucketmap = nullptr;
    sl.grids = w.grid;
    sl.nslots = 1;
    sl.one = rec;
    return sl;
}

// Grid build of a plain call; `periodic` selects the SIR grid.
int plain_grid(const bdm_soa *s, const bdm_params *p, bool periodic, const bdm::Ws &w, hipStream_t st,
               bdm::SlotDev *rec_out) {
    bdm::SlotDev rec = slot_record(p, 0, s->capacity, 0, w.lay.max_boxes, 1, s->diam != nullptr);
    rec.periodic = periodic ? 1 : 0;
    if (periodic) {
        int rc = periodic_boxes(p, w.lay.max_boxes, &rec.nb);
        if (rc) return rc;
    }
    bdm::launch_grid_build(*s, plain_slots(w, rec), s->capacity, false, w, st);
    if (rec_out) *rec_out = rec;
    return hip_check("grid_build launch");
}

bdm::Threshold threshold(double prob) {
    bdm::Threshold t{0, 0};
    if (!(prob > 0.0)) return t;
    if (prob >= 1.0) {
        t.mode = 2;
        return t;
    }
    t.mode = 1;
    t.t = static_cast<uint64_t>(std::ldexp(prob, 64));  // exact scaling, truncation = floor
    return t;
}

int check_sir_params(const bdm_params *p) {
    if (!p) return fail(BDM_EINVAL, "params is NULL");
    if (!(p->r_inf >= 0.0) || !is_fin(p->r_inf)) return fail(BDM_EINVAL, "r_inf must be >= 0");
    if (p->box < p->r_inf) return fail(BDM_EINVAL, "box must be >= r_inf");
    if (!(p->walk >= 0.0) || !(p->walk <= p->L)) return fail(BDM_EINVAL, "walk must be in [0, L]");
    if (std::isnan(p->p_inf) || std::isnan(p->p_rec)) return fail(BDM_EINVAL, "probabilities must not be NaN");
    return BDM_OK;
}

int check_spheroid_params(const bdm_params *p) {
    if (!(p->grow > 0.0) || !is_fin(p->grow)) return fail(BDM_EINVAL, "grow must be > 0");
    if (!(p->div_d > 0.0) || !is_fin(p->div_d)) return fail(BDM_EINVAL, "div_d must be > 0");
    if (!(p->half_cbrt > 0.0) || !(p->half_cbrt < 1.0)) return fail(BDM_EINVAL, "half_cbrt must be in (0, 1)");
    return BDM_OK;
}

int check_oncology_params(const bdm_params *p) {
    if (!(p->p_apo >= 0.0) || !(p->p_apo <= 1.0)) return fail(BDM_EINVAL, "p_apo must be in [0, 1]");
    if (!(p->migrate >= 0.0) || !is_fin(p->migrate)) return fail(BDM_EINVAL, "migrate must be finite and >= 0");
    return BDM_OK;
}

int check_field(const bdm_field *f, bdm::FieldDev *out) {
    if (!f) return fail(BDM_EINVAL, "field is NULL");
    const int32_t lim = 1 << 20;
    if (f->nx < 1 || f->ny < 1 || f->nz < 1 || f->nx > lim || f->ny > lim || f->nz > lim)
        return fail(BDM_EINVAL, "field voxels per axis must be in [1, 2^20]");
    const int64_t V = int64_t(f->nx) * f->ny * f->nz;
    if (V > (int64_t(1) << 30)) return fail(BDM_EINVAL, "field has more than 2^30 voxels");
    if (f->ny > 16 * 65535) return fail(BDM_EINVAL, "field ny must be at most 1048560");  // (launch rows of 16)
    if (!(f->h > 0.0) || !is_fin(f->h) || !is_fin(f->x0) || !is_fin(f->y0) || !is_fin(f->z0))
        return fail(BDM_EINVAL, "field corner must be finite and h > 0");
    if (!f->c || !f->c_next || !f->count) return fail(BDM_EINVAL, "field arrays c, c_next and count are required");
    const char *a = reinterpret_cast<const char *>(f->c), *b = reinterpret_cast<const char *>(f->c_next);
    const size_t bytes = size_t(2 * V) * sizeof(double);
    if (a < b + bytes && b < a + bytes) return fail(BDM_EINVAL, "c and c_next overlap");
    *out = bdm::FieldDev{f->nx, f->ny, f->nz, f->x0, f->y0, f->z0, f->h, V};
    return BDM_OK;
}

int diffusion_coefficients(const bdm_params *p, double h, double *lam, double *kdec) {
    if (!p) return fail(BDM_EINVAL, "params is NULL");
    if (!(p->dt > 0.0) || !is_fin(p->dt)) return fail(BDM_EINVAL, "dt must be > 0");
    *lam = (p->diff_D * p->dt) / (h * h);
    *kdec = p->diff_decay * p->dt;
    if (!(*lam >= 0.0) || !(*lam <= 1.0 / 6.0))
        return fail(BDM_EINVAL, "diff_D*dt/h^2 = %g outside [0, 1/6]", *lam);
    if (!(*kdec >= 0.0) || !(*kdec <= 1.0)) return fail(BDM_EINVAL, "diff_decay*dt = %g outside [0, 1]", *kdec);
    return BDM_OK;
}

int read_grid(const bdm::GridDev *src, bdm::GridDev *dst, hipStream_t st) {
    if (hipMemcpyAsync(dst, src, sizeof *dst, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return hip_check("grid read");
    return BDM_OK;
}

}  // namespace

extern "C" {

size_t bdm_workspace_bytes(int64_t capacity, int64_t max_boxes) {
    bdm::WsLayout lay;
    if (!bdm::ws_layout(capacity, max_boxes, 0, &lay)) return 0;
    return lay.total;
}

int bdm_workspace_init(const bdm_workspace *ws, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_ws(ws, &w);
    if (rc) return rc;
    rc = check_device();
    if (rc) return rc;
    bdm::launch_ws_init(w, as_stream(stream));
    return hip_check("workspace_init launch");
}

int bdm_generate(const bdm_soa *soa, const bdm_gen *gen, void *stream) {
    g_last_error.clear();
    if (!soa || !gen) return fail(BDM_EINVAL, "soa and gen are required");
    if (!soa->n || !soa->x || !soa->y || !soa->z || !soa->id) return fail(BDM_EINVAL, "soa needs n, x, y, z, id");
    if (gen->n < 0 || gen->n > soa->capacity)
        return fail(BDM_EINVAL, "gen n %lld outside [0, capacity]", (long long)gen->n);
    if (gen->n > (int64_t(1) << 32) - 2) return fail(BDM_EINVAL, "at most 2^32 - 2 agents");
    if (gen->kind != BDM_GEN_CUBE && gen->kind != BDM_GEN_BALL && gen->kind != BDM_GEN_SIR &&
        gen->kind != BDM_GEN_SOMA)
        return fail(BDM_EINVAL, "unknown generator kind %d", gen->kind);
    if (!is_fin(gen->L) || !is_fin(gen->dlo) || !is_fin(gen->dhi) || !is_fin(gen->adh))
        return fail(BDM_EINVAL, "generator parameters must be finite");
    if ((gen->kind == BDM_GEN_SIR || gen->kind == BDM_GEN_SOMA) && !soa->state)
        return fail(BDM_EINVAL, "SIR and soma generators need state");
    bdm::GenArgs a{gen->kind, gen->n, gen->L, gen->dlo, gen->dhi, gen->adh, gen->n_infected, gen->seed, gen->salt};
    bdm::launch_generate(*soa, a, as_stream(stream));
    return hip_check("generate launch");
}

int bdm_grid_build(const bdm_soa *soa, const bdm_params *params, const bdm_workspace *ws, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_ws(ws, &w);
    if (rc) return rc;
    if (!params) return fail(BDM_EINVAL, "params is NULL");
    rc = check_soa(soa, w.lay.capacity, false, false);
    if (rc) return rc;
    if (!is_fin(params->box)) return fail(BDM_EINVAL, "box must be finite");
    if (params->skip_static != 0 && params->skip_static != 1) return fail(BDM_EINVAL, "skip_static must be 0 or 1");
    rc = check_skip(soa, params);
    if (rc) return rc;
    return plain_grid(soa, params, params->periodic != 0, w, as_stream(stream), nullptr);
}

int bdm_mech_step(const bdm_soa *soa, const bdm_params *params, const bdm_workspace *ws, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_ws(ws, &w);
    if (rc) return rc;
    rc = check_soa(soa, w.lay.capacity, true, false);
    if (rc) return rc;
    rc = check_mech_params(params);
    if (rc) return rc;
    rc = check_skip(soa, params);
    if (rc) return rc;
    const bdm::SlotDev rec = slot_record(params, 0, soa->capacity, 0, w.lay.max_boxes, 1, true);
    bdm::launch_mech(*soa, plain_slots(w, rec), soa->capacity, params->force_bits, false, w, as_stream(stream));
    return hip_check("mech_step launch");
}

}  // extern "C"

namespace {

int sim_step(const bdm_soa *soa, int32_t model, const bdm_params *params, int64_t step, const bdm_workspace *ws,
             const bdm::TraceOut *trace, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_ws(ws, &w);
    if (rc) return rc;
    if (!params) return fail(BDM_EINVAL, "params is NULL");
    if (step < 0) return fail(BDM_EINVAL, "step must be >= 0");
    hipStream_t st = as_stream(stream);
    switch (model) {
    case BDM_MODEL_MECH:
    case BDM_MODEL_SPHEROID:
    case BDM_MODEL_ONCOLOGY: {
        const bool cells = model != BDM_MODEL_MECH;  // growing cells: the crowded mechanics path
        rc = check_soa(soa, w.lay.capacity, true, false);
        if (rc) return rc;
        rc = check_mech_params(params);
        if (rc) return rc;
        bdm::SlotDev rec = slot_record(params, 0, soa->capacity, 0, w.lay.max_boxes, 1, true);
        if (cells) rec.skip = 0;  // (diameters change every step)
        rc = check_skip(soa, params);
        if (rc && rec.skip) return rc;
        if (cells) {
            rc = check_spheroid_params(params);
            if (rc) return rc;
        }
        if (model == BDM_MODEL_ONCOLOGY) {
            rc = check_oncology_params(params);
            if (rc) return rc;
            bdm::ApoArgs apo{threshold(params->p_apo), params->seed, params->salt, uint64_t(step)};
            if (apo.tapo.mode != 0) bdm::launch_apoptosis(*soa, soa->capacity, apo, w, st);
            rc = hip_check("apoptosis launch");
            if (rc) return rc;
        }
        if (cells) {
            bdm::DivArgs a{params->grow, params->div_d, params->half_cbrt, params->seed, params->salt, uint64_t(step)};
            bdm::launch_grow_divide(*soa, plain_slots(w, rec), soa->capacity, a, w, st);
            rc = hip_check("grow_divide launch");
            if (rc) return rc;
        }
        if (model == BDM_MODEL_ONCOLOGY) {
            bdm::MigArgs mig{params->migrate, params->seed, params->salt, uint64_t(step)};
            bdm::launch_migrate(*soa, soa->capacity, mig, st);
            rc = hip_check("migrate launch");
            if (rc) return rc;
        }
        bdm::launch_grid_build(*soa, plain_slots(w, rec), soa->capacity, cells, w, st, trace == nullptr);
        rc = hip_check("grid_build launch");
        if (rc) return rc;
        bdm::launch_mech(*soa, plain_slots(w, rec), soa->capacity, params->force_bits, cells, w, st, trace);
        return hip_check("mech_step launch");
    }
    case BDM_MODEL_SIR: {
        if (trace) return fail(BDM_EINVAL, "a traced step is a mechanical one (MECH, SPHEROID or ONCOLOGY)");
        rc = check_soa(soa, w.lay.capacity, false, true);
        if (rc) return rc;
        rc = check_sir_params(params);
        if (rc) return rc;
        bdm::SlotDev rec;
        rc = plain_grid(soa, params, true, w, st, &rec);
        if (rc) return rc;
        bdm::SirArgs a{};
        a.L = params->L;
        a.half = 0.5 * params->L;
        a.r2 = params->r_inf * params->r_inf;
        a.walk = params->walk;
        a.tinf = threshold(params->p_inf);
        a.trec = threshold(params->p_rec);
        a.seed = params->seed;
        a.salt = params->salt;
        a.step = uint64_t(step);
        bdm::launch_sir(*soa, plain_slots(w, rec), soa->capacity, a, w, st);
        return hip_check("sir_step launch");
    }
    default:
        return fail(BDM_EINVAL, "unknown model %d", model);
    }
}

}  // namespace

extern "C" {

int bdm_sim_step(const bdm_soa *soa, int32_t model, const bdm_params *params, int64_t step,
                 const bdm_workspace *ws, void *stream) {
    return sim_step(soa, model, params, step, ws, nullptr, stream);
}

int bdm_sim_step_traced(const bdm_soa *soa, int32_t model, const bdm_params *params, int64_t step,
                        const bdm_workspace *ws, uint32_t *counts, uint32_t *hashes, void *stream) {
    g_last_error.clear();
    if (!counts || !hashes) return fail(BDM_EINVAL, "counts and hashes are required");
    const bdm::TraceOut t{counts, hashes};
    return sim_step(soa, model, params, step, ws, &t, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Step without a caller workspace
// ---------------------------------------------------------------------------------------------
// The workspace of bdm_sim_step_noalloc: a static device array, one copy on every device that
// runs the entry point, held until the process ends.  In host code `scratch` only names the
// symbol; its device address on the current device comes from hipGetSymbolAddress, looked up
// once per device and kept in g_scratch_ptr, and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[BDM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the device's first call).
int scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(BDM_ENODEV, "no HIP device");
    if (dev < 0 || dev >= kMaxDevices) return fail(BDM_ENODEV, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int rc = check_device();
        if (rc) return rc;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(BDM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BDM_OK;
}

}  // namespace

extern "C" {

int bdm_sim_step_noalloc(const bdm_soa *soa, int32_t model, const bdm_params *params, int64_t step,
                         int64_t max_boxes, uint32_t *flags, void *stream) {
    g_last_error.clear();
    if (!soa) return fail(BDM_EINVAL, "soa is NULL");
    bdm::WsLayout lay;
    if (!bdm::ws_layout(soa->capacity, max_boxes, 0, &lay))
        return fail(BDM_EINVAL, "capacity %lld / max_boxes %lld out of range", (long long)soa->capacity,
                    (long long)max_boxes);
    if (lay.total > size_t(BDM_NOALLOC_SCRATCH_BYTES))
        return fail(BDM_ENOWS, "capacity %lld and max_boxes %lld need %zu bytes of workspace; the static scratch "
                    "holds %zu", (long long)soa->capacity, (long long)max_boxes, lay.total,
                    size_t(BDM_NOALLOC_SCRATCH_BYTES));
    void *ptr = nullptr;
    int rc = scratch_address(&ptr);
    if (rc) return rc;
    const bdm_workspace ws{ptr, size_t(BDM_NOALLOC_SCRATCH_BYTES), soa->capacity, max_boxes};
    bdm::Ws w;
    rc = get_ws(&ws, &w);
    if (rc) return rc;
    hipStream_t st = as_stream(stream);
    // the previous call's contents stay in the array: start from a cleared grid, histogram and
    // tile order, as bdm_workspace_init leaves a workspace
    bdm::launch_ws_init(w, st);
    rc = hip_check("noalloc workspace init launch");
    if (rc) return rc;
    rc = sim_step(soa, model, params, step, &ws, nullptr, stream);
    if (rc) return rc;
    if (flags) {
        bdm::launch_copy_flags(w, flags, st);
        return hip_check("noalloc flags launch");
    }
    return BDM_OK;
}

int bdm_read_agents(const bdm_soa *soa, double *out_x, double *out_y, double *out_z, double *out_diam,
                    double *out_fx, double *out_fy, double *out_fz, uint8_t *out_state, void *stream) {
    g_last_error.clear();
    if (!soa || !soa->n || !soa->id) return fail(BDM_EINVAL, "soa needs n and id");
    if ((out_x && !soa->x) || (out_y && !soa->y) || (out_z && !soa->z) || (out_diam && !soa->diam) ||
        (out_fx && !soa->fx) || (out_fy && !soa->fy) || (out_fz && !soa->fz) || (out_state && !soa->state))
        return fail(BDM_EINVAL, "an output was requested for an array the soa does not have");
    bdm::ReadOut o{out_x, out_y, out_z, out_diam, out_fx, out_fy, out_fz, out_state};
    bdm::launch_read_agents(*soa, o, as_stream(stream));
    return hip_check("read_agents launch");
}

int bdm_extreme_points(const bdm_soa *soa, const double *dirs, int32_t ndir, uint64_t *work, int32_t *out_slot,
                       void *stream) {
    g_last_error.clear();
    if (!soa || !soa->n || !soa->x || !soa->y || !soa->z) return fail(BDM_EINVAL, "soa positions are required");
    if (soa->capacity < 0 || soa->capacity > INT32_MAX) return fail(BDM_EINVAL, "capacity must be in [0, 2^31)");
    if (ndir < 1 || ndir > BDM_HULL_MAX_DIRS) return fail(BDM_EINVAL, "ndir must be in [1, %d]", BDM_HULL_MAX_DIRS);
    if (!dirs || !work || !out_slot) return fail(BDM_EINVAL, "dirs, work and out_slot are required");
    int rc = check_device();
    if (rc) return rc;
    bdm::launch_extreme_points(*soa, dirs, ndir, reinterpret_cast<unsigned long long *>(work), out_slot,
                               as_stream(stream));
    return hip_check("extreme_points launch");
}

int bdm_hull_candidates(const bdm_soa *soa, const double *planes, int32_t nplane, double tol, int32_t *out_slot,
                        int64_t max_out, int64_t *out_count, void *stream) {
    g_last_error.clear();
    if (!soa || !soa->n || !soa->x || !soa->y || !soa->z) return fail(BDM_EINVAL, "soa positions are required");
    if (soa->capacity < 0 || soa->capacity > INT32_MAX) return fail(BDM_EINVAL, "capacity must be in [0, 2^31)");
    if (nplane < 1 || nplane > BDM_HULL_MAX_PLANES)
        return fail(BDM_EINVAL, "nplane must be in [1, %d]", BDM_HULL_MAX_PLANES);
    if (!(tol >= 0.0) || !is_fin(tol)) return fail(BDM_EINVAL, "tol must be finite and >= 0");
    if (!planes || !out_count || max_out < 0 || (max_out > 0 && !out_slot))
        return fail(BDM_EINVAL, "planes, out_count and (for max_out > 0) out_slot are required");
    int rc = check_device();
    if (rc) return rc;
    bdm::launch_hull_keep(*soa, planes, nplane, tol, out_slot, max_out, out_count, as_stream(stream));
    return hip_check("hull_candidates launch");
}

int bdm_field_init(const bdm_field *field, void *stream) {
    g_last_error.clear();
    bdm::FieldDev f;
    int rc = check_field(field, &f);
    if (rc) return rc;
    rc = check_device();
    if (rc) return rc;
    bdm::launch_field_fill(field->c, field->count, 2 * f.V, as_stream(stream));
    return hip_check("field_init launch");
}

int bdm_diffuse(const bdm_field *field, const bdm_params *params, void *stream) {
    g_last_error.clear();
    bdm::FieldDev f;
    int rc = check_field(field, &f);
    if (rc) return rc;
    double lam = 0.0, kdec = 0.0;
    rc = diffusion_coefficients(params, f.h, &lam, &kdec);
    if (rc) return rc;
    rc = check_device();
    if (rc) return rc;
    bdm::launch_diffuse(f, field->c, field->c_next, lam, kdec, as_stream(stream));
    return hip_check("diffuse launch");
}

int bdm_soma_step(const bdm_soa *soa, const bdm_params *params, const bdm_field *field, const bdm_workspace *ws,
                  void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_ws(ws, &w);
    if (rc) return rc;
    if (!params) return fail(BDM_EINVAL, "params is NULL");
    rc = check_soa(soa, w.lay.capacity, true, true);
    if (rc) return rc;
    rc = check_mech_params(params);
    if (rc) return rc;
    bdm::FieldDev f;
    rc = check_field(field, &f);
    if (rc) return rc;
    double lam = 0.0, kdec = 0.0;
    rc = diffusion_coefficients(params, f.h, &lam, &kdec);
    if (rc) return rc;
    if (!is_fin(params->secrete)) return fail(BDM_EINVAL, "secrete must be finite");
    if (!(params->chemo_speed >= 0.0) || !is_fin(params->chemo_speed))
        return fail(BDM_EINVAL, "chemo_speed must be finite and >= 0");
    hipStream_t st = as_stream(stream);
    bdm::launch_secrete(*soa, soa->capacity, f, field->count, field->c, params->secrete, st);
    bdm::launch_diffuse(f, field->c, field->c_next, lam, kdec, st);
    bdm::launch_chemotaxis(*soa, soa->capacity, f, field->c_next, params->chemo_speed, st);
    rc = hip_check("substance launches");
    if (rc) return rc;
    bdm::SlotDev rec = slot_record(params, 0, soa->capacity, 0, w.lay.max_boxes, 1, true);
    rec.skip = 0;
    bdm::launch_grid_build(*soa, plain_slots(w, rec), soa->capacity, false, w, st);
    rc = hip_check("grid_build launch");
    if (rc) return rc;
    bdm::launch_mech(*soa, plain_slots(w, rec), soa->capacity, params->force_bits, false, w, st);
    return hip_check("mech_step launch");
}

int bdm_geom_step(const bdm_soa *soa, const bdm_cylinders *cyl, const bdm_params *params, const bdm_workspace *ws,
                  uint32_t *counts, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_ws(ws, &w);
    if (rc) return rc;
    if (!params) return fail(BDM_EINVAL, "params is NULL");
    rc = check_soa(soa, w.lay.capacity, true, true);
    if (rc) return rc;
    rc = check_mech_params(params);
    if (rc) return rc;
    if (params->force_bits != 64) return fail(BDM_EINVAL, "the cylinder step uses the binary64 law (force_bits 64)");
    if (!cyl || !cyl->px || !cyl->py || !cyl->pz || !cyl->dc)
        return fail(BDM_EINVAL, "cylinder arrays px, py, pz and dc are required");
    hipStream_t st = as_stream(stream);
    const bdm::CylIn in{cyl->px, cyl->py, cyl->pz, cyl->dc};
    bdm::launch_geom_reach(*soa, soa->capacity, in, st);
    bdm::SlotDev rec = slot_record(params, 0, soa->capacity, 0, w.lay.max_boxes, 1, true);
    rec.skip = 0;
    bdm::launch_grid_build(*soa, plain_slots(w, rec), soa->capacity, false, w, st);
    rc = hip_check("grid_build launch");
    if (rc) return rc;
    const bdm::GeomArgs a{params->k, params->gamma, params->dt, params->max_disp, soa->capacity};
    bdm::launch_geom(*soa, in, a, w, counts, st);
    return hip_check("geom_step launch");
}

int bdm_status(const bdm_workspace *ws, uint32_t *flags, int32_t clear, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_ws(ws, &w);
    if (rc) return rc;
    if (!flags) return fail(BDM_EINVAL, "flags is NULL");
    hipStream_t st = as_stream(stream);
    if (hipMemcpyAsync(flags, &w.grid->flags, sizeof(uint32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return hip_check("status read");
    if (clear) {
        if (hipMemsetAsync(&w.grid->flags, 0, sizeof(uint32_t), st) != hipSuccess) return hip_check("status clear");
    }
    return BDM_OK;
}

int bdm_sir_counts(const bdm_workspace *ws, int64_t *counts, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_ws(ws, &w);
    if (rc) return rc;
    if (!counts) return fail(BDM_EINVAL, "counts is NULL");
    bdm::GridDev g;
    rc = read_grid(w.grid, &g, as_stream(stream));
    if (rc) return rc;
    for (int i = 0; i < 3; ++i) counts[i] = int64_t(g.sir_counts[i]);
    return BDM_OK;
}

int bdm_grid_info(const bdm_workspace *ws, bdm_grid_desc *desc, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_ws(ws, &w);
    if (rc) return rc;
    if (!desc) return fail(BDM_EINVAL, "desc is NULL");
    bdm::GridDev g;
    rc = read_grid(w.grid, &g, as_stream(stream));
    if (rc) return rc;
    desc->b = g.b;
    for (int i = 0; i < 3; ++i) {
        desc->cmin[i] = g.cmin[i];
        desc->dims[i] = g.dims[i];
    }
    desc->nboxes = g.nboxes;
    desc->n = g.n;
    desc->valid = g.valid;
    desc->flags = g.flags;
    desc->skipped = g.skipped;
    return BDM_OK;
}

int bdm_grid_export(const bdm_workspace *ws, uint32_t *key, uint32_t *order, uint32_t *start, void *stream) {
    bdm_grid_desc d;
    int rc = bdm_grid_info(ws, &d, stream);
    if (rc) return rc;
    if (!d.valid) return fail(BDM_EINVAL, "no valid grid in the workspace");
    bdm::Ws w;
    get_ws(ws, &w);
    hipStream_t st = as_stream(stream);
    size_t n = size_t(d.n);
    if (key && n && hipMemcpyAsync(key, w.key, 4 * n, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return hip_check("grid_export key");
    if (order && n && hipMemcpyAsync(order, w.ids, 4 * n, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return hip_check("grid_export order");
    if (start) {
        if (hipMemcpyAsync(start, w.start, 4 * (size_t(d.nboxes) + 1), hipMemcpyDeviceToDevice, st) != hipSuccess)
            return hip_check("grid_export start");
        bdm::launch_mask_starts(start, d.nboxes + 1, st);  // (the stationary-skip marks)
    }
    if (hipStreamSynchronize(st) != hipSuccess) return hip_check("grid_export sync");
    return BDM_OK;
}

int bdm_contacts(const bdm_workspace *ws, const bdm_params *params, uint32_t *counts, const int64_t *offsets,
                 uint32_t *ids, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_ws(ws, &w);
    if (rc) return rc;
    if (!params || !counts) return fail(BDM_EINVAL, "params and counts are required");
    if (ids && !offsets) return fail(BDM_EINVAL, "ids need offsets");
    bdm::ContactArgs a{};
    if (params->periodic) {
        a.mode = 2;
        a.L = params->L;
        a.half = 0.5 * params->L;
        a.r2 = params->r_inf * params->r_inf;
    } else {
        if (params->force_bits != 32 && params->force_bits != 64) return fail(BDM_EINVAL, "force_bits must be 32 or 64");
        a.mode = params->force_bits == 32 ? 1 : 0;
    }
    const bdm::SlotDev rec = slot_record(params, 0, w.lay.capacity, 0, w.lay.max_boxes, 1, true);
    bdm::launch_contacts(a, plain_slots(w, rec), w, counts, offsets, ids, as_stream(stream));
    return hip_check("contacts launch");
}

int bdm_fp_probe(const double *a, const double *b, int64_t n, double *out_sqrt, double *out_div,
                 float *out_sqrtf, float *out_divf, void *stream) {
    g_last_error.clear();
    if (n < 0 || (n > 0 && (!a || !b))) return fail(BDM_EINVAL, "fp_probe needs a and b");
    if (n == 0) return BDM_OK;
    bdm::launch_fp_probe(a, b, n, out_sqrt, out_div, out_sqrtf, out_divf, as_stream(stream));
    return hip_check("fp_probe launch");
}

// ---------------------------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------------------------
size_t bdm_batch_workspace_bytes(int64_t capacity, int64_t max_boxes, int32_t slots) {
    bdm::WsLayout lay;
    if (slots < 1 || !bdm::ws_layout(capacity, max_boxes, slots, &lay)) return 0;
    return lay.total;
}

int bdm_batch_init(const bdm_batch *b, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_batch(b, &w);
    if (rc) return rc;
    rc = check_device();
    if (rc) return rc;
    bdm::launch_ws_init(w, as_stream(stream));
    return hip_check("batch_init launch");
}

int bdm_batch_set_slot(const bdm_batch *b, int32_t slot, int64_t agent_off, int64_t capacity, int64_t box_off,
                       int64_t max_boxes, int64_t steps, const bdm_params *p, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_batch(b, &w);
    if (rc) return rc;
    if (slot < 0 || slot >= b->slots) return fail(BDM_EINVAL, "slot %d outside [0, %d)", slot, b->slots);
    if (agent_off < 0 || agent_off % BDM_SLOT_ALIGN != 0)
        return fail(BDM_EINVAL, "agent_off must be a non-negative multiple of %d", BDM_SLOT_ALIGN);
    if (capacity < 1 || agent_off + capacity > b->capacity)
        return fail(BDM_EINVAL, "slot range [%lld, %lld) outside the batch", (long long)agent_off,
                    (long long)(agent_off + capacity));
    if (box_off % BDM_BOX_ALIGN != 0)
        return fail(BDM_EINVAL, "box_off must be a multiple of %d", BDM_BOX_ALIGN);
    if (box_off < 0 || max_boxes < 1 || box_off + max_boxes > b->max_boxes)
        return fail(BDM_EINVAL, "slot boxes [%lld, %lld) outside the batch", (long long)box_off,
                    (long long)(box_off + max_boxes));
    if (steps < 0) return fail(BDM_EINVAL, "steps must be >= 0");
    rc = check_mech_params(p);
    if (rc) return rc;
    bdm::SlotDev rec = slot_record(p, agent_off, capacity, box_off, max_boxes, steps, true);
    rec.skip = 0;  // (the batched step does not skip stationary agents)
    const int64_t first = agent_off / bdm::kBlock;
    const int64_t ntile = (agent_off + capacity + bdm::kBlock - 1) / bdm::kBlock - first;
    bdm::launch_set_slot(w, slot, rec, first, ntile, slot, as_stream(stream));
    return hip_check("batch_set_slot launch");
}

int bdm_batch_clear_slot(const bdm_batch *b, int32_t slot, int64_t agent_off, int64_t capacity, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_batch(b, &w);
    if (rc) return rc;
    if (slot < 0 || slot >= b->slots) return fail(BDM_EINVAL, "slot %d outside [0, %d)", slot, b->slots);
    if (agent_off < 0 || agent_off % BDM_SLOT_ALIGN != 0 || capacity < 0 || agent_off + capacity > b->capacity)
        return fail(BDM_EINVAL, "slot range outside the batch or misaligned");
    bdm::SlotDev rec{};
    const int64_t first = agent_off / bdm::kBlock;
    const int64_t ntile = (agent_off + capacity + bdm::kBlock - 1) / bdm::kBlock - first;
    bdm::launch_set_slot(w, slot, rec, first, ntile, -1, as_stream(stream));
    return hip_check("batch_clear_slot launch");
}

}  // extern "C"

namespace {

int batch_step(const bdm_soa *packed, const bdm_batch *b, const bdm::TraceOut *trace, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_batch(b, &w);
    if (rc) return rc;
    rc = check_soa(packed, w.lay.capacity, true, false);
    if (rc) return rc;
    if (packed->capacity != b->capacity) return fail(BDM_EINVAL, "packed soa capacity must equal the batch capacity");
    hipStream_t st = as_stream(stream);
    bdm::Slots sl{};
    sl.table = w.slots;
    sl.tilemap = w.tilemap;
    sl.bucketmap = w.bucketmap;
    sl.grids = w.grid;
    sl.nslots = b->slots;
    sl.grid_cap = b->grid_cap;
    bdm::launch_grid_build(*packed, sl, b->capacity, false, w, st);
    bdm::launch_mech(*packed, sl, b->capacity, 0, false, w, st, trace);
    bdm::launch_batch_advance(w, st);
    return hip_check("batch_step launch");
}

}  // namespace

extern "C" {

int bdm_batch_step(const bdm_soa *packed, const bdm_batch *b, void *stream) {
    return batch_step(packed, b, nullptr, stream);
}

int bdm_batch_step_traced(const bdm_soa *packed, const bdm_batch *b, uint32_t *counts, uint32_t *hashes,
                          void *stream) {
    g_last_error.clear();
    if (!counts || !hashes) return fail(BDM_EINVAL, "counts and hashes are required");
    const bdm::TraceOut t{counts, hashes};
    return batch_step(packed, b, &t, stream);
}

int bdm_batch_slot_status(const bdm_batch *b, int32_t slot, uint32_t *flags, int64_t *steps_left, void *stream) {
    g_last_error.clear();
    bdm::Ws w;
    int rc = get_batch(b, &w);
    if (rc) return rc;
    if (slot < 0 || slot >= b->slots) return fail(BDM_EINVAL, "slot %d outside [0, %d)", slot, b->slots);
    hipStream_t st = as_stream(stream);
    bdm::GridDev g;
    bdm::SlotDev s;
    if (hipMemcpyAsync(&g, &w.grid[slot], sizeof g, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(&s, &w.slots[slot], sizeof s, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return hip_check("batch_slot_status read");
    if (flags) *flags = g.flags;
    if (steps_left) *steps_left = s.steps_left;
    return BDM_OK;
}

const char *bdm_strerror(int code) {
    switch (code) {
    case BDM_OK: return "ok";
    case BDM_EINVAL: return "invalid argument";
    case BDM_ENOWS: return "workspace missing or too small";
    case BDM_EHIP: return "HIP runtime error";
    case BDM_ENODEV: return "no usable gfx950 device";
    default: return "unknown error";
    }
}

const char *bdm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
