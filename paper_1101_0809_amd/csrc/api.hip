// api.hip -- the C ABI declared in include/pic.h: validation, buffer
// carve-up, and the step schedule (B half step, particle kernel per mobile
// species, B half step, E update, periodic sort).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include <algorithm>

#include "boundary.h"
#include "pic_internal.h"

namespace pic {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

namespace {

thread_local std::string g_tls_err;

int fail(Ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    else g_tls_err = msg;
    return code;
}

int hip_fail(Ctx* c, hipError_t e, const char* where)
{
    return fail(c, PIC_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

int tile_of(int dims) { return dims == 3 ? kTile3 : kTile2; }

// Fill the kernel constants; returns PIC_OK or an error code with message.
int make_grid(const pic_grid_desc* g, GridK* k, std::string* msg)
{
    if (!g) {
        *msg = "null grid description";
        return PIC_EINVAL;
    }
    if (g->dims != 2 && g->dims != 3) {
        *msg = "dims must be 2 or 3";
        return PIC_EINVAL;
    }
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) {
        *msg = "cell counts must be >= 1";
        return PIC_EINVAL;
    }
    if (g->dims == 2 && g->nz != 1) {
        *msg = "dims == 2 requires nz == 1";
        return PIC_EINVAL;
    }
    if (g->precision != PIC_FP64 && g->precision != PIC_FP32C) {
        *msg = "precision must be PIC_FP64 or PIC_FP32C";
        return PIC_EINVAL;
    }
    if (g->order != 1 && g->order != 2) {
        *msg = "order must be 1 or 2 (alternating order 1 1/2 or 2 1/2)";
        return PIC_EINVAL;
    }
    if (g->order == 2 && g->precision != PIC_FP64) {
        *msg = "alternating order 2 1/2 is FP64 only";
        return PIC_EINVAL;
    }
    if (g->sort_every < 0) {
        *msg = "sort_every must be >= 0";
        return PIC_EINVAL;
    }
    if (g->interp != 0 && g->interp != 1) {
        *msg = "interp must be 0 (alternating order) or 1 (conventional, Eq. wrong1)";
        return PIC_EINVAL;
    }
    if (g->interp == 1 && (g->order != 1 || g->precision != PIC_FP64)) {
        *msg = "the conventional interpolation runs at order 1 in FP64 only";
        return PIC_EINVAL;
    }
    if (!(g->dx > 0) || !(g->dy > 0) || !(g->dz > 0) || !(g->dt > 0) || !(g->c > 0)) {
        *msg = "dx, dy, dz, dt and c must be positive";
        return PIC_EINVAL;
    }
    if (g->precision == PIC_FP32C && (g->nx > 2048 || g->ny > 2048 || g->nz > 1024)) {
        *msg = "FP32 mode packs the cell as 11+11+10 bits: nx, ny <= 2048, nz <= 1024";
        return PIC_EINVAL;
    }
    const int T = tile_of(g->dims);
    k->dims = g->dims;
    k->n[0] = g->nx;
    k->n[1] = g->ny;
    k->n[2] = g->nz;
    k->tile[0] = T;
    k->tile[1] = T;
    k->tile[2] = g->dims == 3 ? T : 1;
    for (int a = 0; a < 3; ++a) k->nt[a] = (k->n[a] + k->tile[a] - 1) / k->tile[a];
    const int64_t ntiles = (int64_t)k->nt[0] * k->nt[1] * k->nt[2];
    const int64_t tpd = (int64_t)k->tile[0] * k->tile[1] * k->tile[2];
    if (ntiles * tpd >= (int64_t)UINT32_MAX || ntiles > (1 << 30)) {
        *msg = "grid too large for 32-bit sort keys";
        return PIC_EINVAL;
    }
    k->ntiles = (int)ntiles;
    k->ncell = (int64_t)g->nx * g->ny * g->nz;
    const double h[3] = {g->dx, g->dy, g->dz};
    double cfl2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        k->cfl[a] = g->c * g->dt / h[a];
        k->half_cfl[a] = 0.5 * k->cfl[a];
        k->inv_h[a] = 1.0 / h[a];
        if (k->n[a] > 1 && a < g->dims) cfl2 += k->cfl[a] * k->cfl[a];
        if (k->cfl[a] >= 1.0) {
            *msg = "c dt / d >= 1 on some axis: a particle could cross more than one cell";
            return PIC_ECFL;
        }
    }
    if (cfl2 >= 1.0) {
        char buf[160];
        snprintf(buf, sizeof buf, "Courant condition violated: sum (c dt/d)^2 = %.6g >= 1", cfl2);
        *msg = buf;
        return PIC_ECFL;
    }
    k->dt = g->dt;
    k->c = g->c;
    for (int a = 0; a < 3; ++a) k->bext[a] = g->bext[a];
    const double V = g->dx * g->dy * g->dz;
    k->inv_vol = 1.0 / V;
    for (int a = 0; a < 3; ++a) k->jscale[a] = -0.25 * h[a] / g->dt / V;
    k->fourpidt = 4.0 * kPi * g->dt;
    if (g->src_kind != 0 && g->src_kind != 1) {
        *msg = "src_kind must be 0 or 1";
        return PIC_EINVAL;
    }
    if (g->src_kind == 1 && (g->src_plane < 2 || g->src_plane > g->nx - 2 || !(g->src_ramp >= 0.0)
                             || !isfinite(g->src_amp) || !isfinite(g->src_omega))) {
        *msg = "plane-wave source needs 2 <= src_plane <= nx - 2, finite amplitude and omega, ramp >= 0";
        return PIC_EINVAL;
    }
    k->src_kind = g->src_kind;
    k->src_plane = g->src_plane;
    k->src_amp = g->src_amp;
    k->src_omega = g->src_omega;
    k->src_ramp = g->src_ramp;
    k->aux = nullptr;
    if (g->field_form != 0 && g->field_form != 1) {
        *msg = "field_form must be 0 (B) or 1 (vector potential)";
        return PIC_EINVAL;
    }
    if (g->xbc != 0 && g->xbc != 1) {
        *msg = "xbc must be 0 (periodic) or 1 (open)";
        return PIC_EINVAL;
    }
    if (g->xbc == 1 && (g->nx < 8 || g->order != 1 || g->interp != 0 || g->field_form != 0 ||
                        (g->src_kind == 1 && g->src_plane > g->nx - 3))) {
        *msg = "the open x boundary needs nx >= 8, the alternating order 1 1/2 with B carried, "
               "and a source plane <= nx - 3";
        return PIC_EINVAL;
    }
    if (g->field_form == 1 && g->src_kind != 0) {
        *msg = "the vector-potential form does not carry the plane-wave source";
        return PIC_EINVAL;
    }
    k->field_form = g->field_form;
    return PIC_OK;
}

size_t workspace_bytes(const GridK& k, uint32_t nkeys)
{
    size_t b = 0;
    b += 3 * align_up((size_t)k.ncell * 8, kAlign);                     // rho_bg, r0, rho_m
    b += align_up(((size_t)nkeys + 1) * 4, kAlign);                      // hist
    b += align_up(((size_t)nkeys / 1024 + 2) * 4, kAlign);               // scan partials
    b += align_up(diag_partials_doubles(kMaxSpecies) * 8, kAlign);       // reductions
    b += align_up(8 * sizeof(unsigned long long), kAlign);               // counters
    b += align_up(3 * (size_t)k.ncell * 8, kAlign);                      // B^n for the particles
    b += align_up(3 * (size_t)k.ncell * 8, kAlign);                      // adjoint scratch
    if (k.field_form == 1) b += align_up(3 * (size_t)k.ncell * 8, kAlign);  // vector potential
    b += align_up((size_t)k.ntiles * 4, kAlign);                         // migrant bucket counters
    b += align_up(2 * (size_t)PIC_AUX * 8, kAlign);                      // source line (last)
    return b;
}

size_t particle_copy_bytes(int precision, int64_t cap)
{
    const size_t C = (size_t)cap;
    if (precision == PIC_FP64)  // pos 3, mom 3, weight, id: 8 arrays of 8 bytes
        return 8 * align_up(C * 8, kAlign);
    // cell, pos 3, mom 3, weight (4 bytes each) + id (8 bytes)
    return 8 * align_up(C * 4, kAlign) + align_up(C * 8, kAlign);
}

size_t particle_bytes(const GridK& k, int precision, int64_t cap)
{
    const size_t C = (size_t)cap;
    return 2 * particle_copy_bytes(precision, cap) + 4 * align_up(C * 4, kAlign) +
           align_up(((size_t)k.ntiles + 1) * 8, kAlign);
}

void carve_copy(char*& p, int precision, int64_t cap, PartArrays* a)
{
    const size_t C = (size_t)cap;
    const size_t es = precision == PIC_FP64 ? 8 : 4;
    auto take = [&](size_t bytes) {
        char* r = p;
        p += align_up(bytes, kAlign);
        return (void*)r;
    };
    for (int ax = 0; ax < 3; ++ax) a->pos[ax] = take(C * es);
    for (int ax = 0; ax < 3; ++ax) a->mom[ax] = take(C * es);
    a->weight = take(C * es);
    a->cell = precision == PIC_FP64 ? nullptr : (uint32_t*)take(C * 4);
    a->id = (int64_t*)take(C * 8);
}

__global__ void k_zero_counters(unsigned long long* p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// Clear counters with a kernel rather than a memset node, so that a step can
// be captured into a HIP graph and replayed.
hipError_t zero_counters(unsigned long long* p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t ensure_sorted(Ctx& c, hipStream_t s)
{
    for (int i = 0; i < c.nsp; ++i) {
        Species& sp = c.sp[i];
        if (sp.d.mobile && !sp.sorted) {
            hipError_t e = launch_sort(c, sp, s);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t ensure_r0(Ctx& c, hipStream_t s)
{
    if (c.r0_valid) return hipSuccess;
    hipError_t e = launch_capture_r0(c, s);
    if (e == hipSuccess) c.r0_valid = true;
    return e;
}

}  // namespace
}  // namespace pic

using namespace pic;

struct pic_ctx {
    Ctx c;
    // event timing (pic_timing_start / pic_timing_stop): 5 events per step
    std::vector<hipEvent_t> ev;
    int timing_cap = 0;
    int timing_used = 0;
    ~pic_ctx()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

extern "C" {

const char* pic_version(void) { return "pic-aoi-gfx950 0.1"; }

const char* pic_last_error(const pic_ctx* ctx)
{
    if (!ctx) return g_tls_err.c_str();
    return ctx->c.err.c_str();
}

int pic_query_sizes(const pic_grid_desc* g, int64_t cap, pic_sizes* out)
{
    if (!out || cap < 0) return fail(nullptr, PIC_EINVAL, "null output or negative capacity");
    GridK k{};
    std::string msg;
    int rc = make_grid(g, &k, &msg);
    if (rc != PIC_OK) return fail(nullptr, rc, msg);
    const uint32_t nkeys = (uint32_t)(k.ntiles * (int64_t)k.tile[0] * k.tile[1] * k.tile[2]);
    out->field_bytes = (size_t)9 * k.ncell * 8;
    out->workspace_bytes = workspace_bytes(k, nkeys);
    out->particle_bytes = particle_bytes(k, g->precision, cap);
    return PIC_OK;
}

int pic_init_grid(const pic_grid_desc* g, void* fields, size_t field_bytes, void* workspace,
                  size_t ws_bytes, pic_ctx** out)
{
    if (!out) return fail(nullptr, PIC_EINVAL, "null output pointer");
    *out = nullptr;
    GridK k{};
    std::string msg;
    int rc = make_grid(g, &k, &msg);
    if (rc != PIC_OK) return fail(nullptr, rc, msg);
    if (!fields || !workspace) return fail(nullptr, PIC_EINVAL, "null field or workspace buffer");
    const uint32_t nkeys = (uint32_t)(k.ntiles * (int64_t)k.tile[0] * k.tile[1] * k.tile[2]);
    if (field_bytes < (size_t)9 * k.ncell * 8 || ws_bytes < workspace_bytes(k, nkeys))
        return fail(nullptr, PIC_ESIZE, "field or workspace buffer smaller than pic_query_sizes");
    pic_ctx* ctx = new (std::nothrow) pic_ctx;
    if (!ctx) return fail(nullptr, PIC_EINVAL, "out of host memory");
    Ctx& c = ctx->c;
    c.g = *g;
    c.k = k;
    c.fields = (double*)fields;
    c.ws = (char*)workspace;
    c.ws_bytes = ws_bytes;
    c.nkeys = nkeys;
    char* p = c.ws;
    auto take = [&](size_t bytes) {
        char* r = p;
        p += align_up(bytes, kAlign);
        return (void*)r;
    };
    c.rho_bg = (double*)take((size_t)k.ncell * 8);
    c.r0 = (double*)take((size_t)k.ncell * 8);
    c.rho_m = (double*)take((size_t)k.ncell * 8);
    c.hist = (uint32_t*)take(((size_t)nkeys + 1) * 4);
    c.scan_part = (uint32_t*)take(((size_t)nkeys / 1024 + 2) * 4);
    c.red = (double*)take(diag_partials_doubles(kMaxSpecies) * 8);
    c.counters = (unsigned long long*)take(8 * sizeof(unsigned long long));
    c.bn = (double*)take(3 * (size_t)k.ncell * 8);
    c.adj = (double*)take(3 * (size_t)k.ncell * 8);
    if (k.field_form == 1) c.avec = (double*)take(3 * (size_t)k.ncell * 8);
    c.mig_n = (unsigned int*)take((size_t)k.ntiles * 4);
    c.k.aux = (double*)take(2 * (size_t)PIC_AUX * 8);  // last: its place is documented
    hipError_t e = hipMemset(c.rho_bg, 0, (size_t)k.ncell * 8);
    if (e == hipSuccess && c.avec) {  // A = 0 and B = curl_h A = 0
        e = hipMemset(c.avec, 0, 3 * (size_t)k.ncell * 8);
        if (e == hipSuccess) e = hipMemset(c.fields + 3 * k.ncell, 0, 3 * (size_t)k.ncell * 8);
    }
    if (e == hipSuccess) e = hipMemset(c.k.aux, 0, 2 * (size_t)PIC_AUX * 8);
    if (e == hipSuccess) e = hipMemset(c.counters, 0, 8 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(c.mig_n, 0, (size_t)k.ntiles * 4);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete ctx;
        return fail(nullptr, PIC_EDEVICE, std::string("init: ") + hipGetErrorString(e));
    }
    *out = ctx;
    return PIC_OK;
}

int pic_add_species(pic_ctx* ctx, const pic_species_desc* s, void* buffer, size_t bytes,
                    int* species)
{
    if (!ctx || !s || !species) return fail(ctx ? &ctx->c : nullptr, PIC_EINVAL, "null argument");
    Ctx& c = ctx->c;
    if (c.nsp >= kMaxSpecies) return fail(&c, PIC_ESTATE, "at most 4 species");
    if (!(s->m > 0) || !isfinite(s->q) || s->capacity < 0 || s->capacity > (int64_t)UINT32_MAX ||
        s->reserved != 0)
        return fail(&c, PIC_EINVAL, "species needs m > 0, finite q, 0 <= capacity < 2^32, reserved 0");
    Species& sp = c.sp[c.nsp];
    sp = Species{};
    sp.d = *s;
    if (s->mobile) {
        const size_t need = particle_bytes(c.k, c.g.precision, s->capacity);
        if (!buffer || bytes < need)
            return fail(&c, PIC_ESIZE, "particle buffer smaller than pic_query_sizes");
        sp.buf = (char*)buffer;
        sp.bytes = bytes;
        char* p = sp.buf;
        carve_copy(p, c.g.precision, s->capacity, &sp.cur);
        carve_copy(p, c.g.precision, s->capacity, &sp.alt);
        sp.key = (uint32_t*)p;
        p += align_up((size_t)s->capacity * 4, kAlign);
        sp.rank = (uint32_t*)p;
        p += align_up((size_t)s->capacity * 4, kAlign);
        sp.dest = (uint32_t*)p;
        p += align_up((size_t)s->capacity * 4, kAlign);
        sp.src = (uint32_t*)p;
        p += align_up((size_t)s->capacity * 4, kAlign);
        sp.tile_start = (int64_t*)p;
    }
    *species = c.nsp++;
    return PIC_OK;
}

int pic_load_particles(pic_ctx* ctx, int species, int64_t n, const double* x, const double* w,
                       const double* weight, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    if (species < 0 || species >= c.nsp) return fail(&c, PIC_EINVAL, "bad species index");
    if (n < 0) return fail(&c, PIC_EINVAL, "negative count");
    if (n == 0) return PIC_OK;
    if (!x || !weight || (!w && c.sp[species].d.mobile))
        return fail(&c, PIC_EINVAL, "null particle array");
    hipStream_t s = (hipStream_t)stream;
    Species& sp = c.sp[species];
    hipError_t e = zero_counters(c.counters, 1, s);
    if (e != hipSuccess) return hip_fail(&c, e, "load");
    if (sp.d.mobile) {
        if (sp.n + n > sp.d.capacity) return fail(&c, PIC_ESIZE, "species capacity exceeded");
        e = launch_load(c, sp, n, x, w, weight, s);
    } else {
        e = launch_rho_raw(c, x, weight, sp.d.q, n, c.rho_bg, s);
    }
    if (e != hipSuccess) return hip_fail(&c, e, "load");
    unsigned long long bad = 0;
    e = hipMemcpyAsync(&bad, c.counters, sizeof bad, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(&c, e, "load");
    if (sp.d.mobile) {
        if (bad) return fail(&c, PIC_ERANGE, "particle positions outside [0, N), or bad weights");
        sp.n += n;
        sp.sorted = false;
    }
    c.r0_valid = false;
    return PIC_OK;
}

int pic_step(pic_ctx* ctx, int nsteps, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    if (nsteps < 0) return fail(&c, PIC_EINVAL, "negative step count");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = ensure_sorted(c, s);
    if (e == hipSuccess) e = ensure_r0(c, s);
    if (e != hipSuccess) return hip_fail(&c, e, "step setup");
    // fallback statistics of this call (pic_last_fallback_fraction), zeroed
    // by the first field kernel of the call
    if (nsteps == 0) {
        e = zero_counters(c.counters + 1, 3, s);
        if (e != hipSuccess) return hip_fail(&c, e, "step");
    }
    for (int it = 0; it < nsteps; ++it) {
        const bool timed = ctx->timing_used < ctx->timing_cap;
        hipEvent_t* ev = timed ? &ctx->ev[5 * (size_t)ctx->timing_used] : nullptr;
        auto mark = [&](int k) {
            if (timed && e == hipSuccess) e = hipEventRecord(ev[k], s);
        };
        // both B half steps use E^n: one kernel writes B^n (for the particles)
        // to the workspace and B^{n+1/2} in place
        mark(0);
        if (e == hipSuccess)
            e = c.k.field_form == 1
                    ? launch_field_half_a_pair(c, s, it == 0 ? c.counters + 1 : nullptr, it == 0 ? 3 : 0)
                    : launch_field_half_b_pair(c, s, it == 0 ? c.counters + 1 : nullptr, it == 0 ? 3 : 0);
        mark(1);
        for (int i = 0; i < c.nsp && e == hipSuccess; ++i)
            if (c.sp[i].d.mobile) e = launch_particle_step(c, c.sp[i], s);
        if (c.g.xbc == 1)  // after every species' current of the step is deposited
            for (int i = 0; i < c.nsp && e == hipSuccess; ++i)
                if (c.sp[i].d.mobile) e = launch_absorb(c, c.sp[i], s);
        mark(2);
        if (e == hipSuccess) e = launch_field_update_e(c, s, c.step);
        mark(3);
        if (e != hipSuccess) return hip_fail(&c, e, "step");
        ++c.step;
        ++c.since_sort;
        if (c.g.sort_every > 0 && c.since_sort >= c.g.sort_every) {
            for (int i = 0; i < c.nsp && e == hipSuccess; ++i)
                if (c.sp[i].d.mobile) e = launch_sort(c, c.sp[i], s);
            if (e != hipSuccess) return hip_fail(&c, e, "sort");
            c.since_sort = 0;
        }
        mark(4);
        if (e != hipSuccess) return hip_fail(&c, e, "step timing");
        if (timed) ++ctx->timing_used;
    }
    return PIC_OK;
}

int pic_deposit_J(pic_ctx* ctx, const double* x0, const double* x1, const double* charge,
                  int64_t n, double* J_out, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    if (n < 0 || (n > 0 && (!x0 || !x1 || !charge || !J_out)))
        return fail(&c, PIC_EINVAL, "null array or negative count");
    hipError_t e = launch_deposit_only(c, x0, x1, charge, n, J_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(&c, e, "deposit_J");
    return PIC_OK;
}

int pic_field_solve(pic_ctx* ctx, int what, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (c.k.field_form != 0) return fail(&c, PIC_ESTATE, "field_solve advances B; this context carries A");
    if (c.g.xbc != 0)
        return fail(&c, PIC_ESTATE, "the open x walls need whole steps (pic_step); field_solve is periodic");
    if (what == PIC_B_HALF) {
        e = launch_field_half_b(c, s);
    } else if (what == PIC_E_FULL) {
        e = launch_field_half_b(c, s);
        if (e == hipSuccess) e = launch_field_update_e(c, s, c.step);
    } else {
        return fail(&c, PIC_EINVAL, "what must be PIC_B_HALF or PIC_E_FULL");
    }
    if (e != hipSuccess) return hip_fail(&c, e, "field_solve");
    return PIC_OK;
}

static int adjoint_ready(Ctx& c)
{
    if (c.g.precision != PIC_FP64) return fail(&c, PIC_EINVAL, "the adjoint is FP64 only");
    if (c.k.src_kind != 0) return fail(&c, PIC_EINVAL, "the adjoint does not cover the plane-wave source");
    if (c.k.field_form != 0) return fail(&c, PIC_EINVAL, "the adjoint covers the B form only");
    if (c.g.xbc != 0) return fail(&c, PIC_EINVAL, "the adjoint covers periodic boxes only");
    if (c.g.order != 1 || c.g.interp != 0)
        return fail(&c, PIC_EINVAL, "the adjoint covers the alternating order 1 1/2 only");
    if (c.k.ncell * (int64_t)sizeof(double) >= ((int64_t)1 << 32))
        return fail(&c, PIC_EINVAL, "the adjoint needs one field plane below 4 GiB (fewer than 2^29 cells)");
    return PIC_OK;
}

int pic_adjoint_seed_field_energy(pic_ctx* ctx, double* lam_fields, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    if (!lam_fields) return fail(&c, PIC_EINVAL, "null adjoint field buffer");
    const int r = adjoint_ready(c);
    if (r != PIC_OK) return r;
    hipError_t e = launch_adjoint_seed(c, lam_fields, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(&c, e, "adjoint_seed_field_energy");
    return PIC_OK;
}

static int adjoint_step_common(pic_ctx* ctx, const void* record, size_t record_bytes, bool by_id,
                               double* lam_fields, double* const* lam_x, double* const* lam_w, double* lam_bext,
                               void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    if (!lam_fields || !lam_bext || !lam_x || !lam_w) return fail(&c, PIC_EINVAL, "null adjoint buffer");
    const int r = adjoint_ready(c);
    if (r != PIC_OK) return r;
    for (int i = 0; i < c.nsp; ++i)
        if (c.sp[i].d.mobile && c.sp[i].n > 0 && (!lam_x[i] || !lam_w[i]))
            return fail(&c, PIC_EINVAL, "null particle adjoint of a mobile species");
    if (record && record_bytes < adjoint_record_bytes(c))
        return fail(&c, PIC_ESIZE, "record smaller than pic_adjoint_record_bytes");
    hipError_t e = launch_adjoint_step(c, record, by_id, lam_fields, lam_x, lam_w, lam_bext, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(&c, e, "adjoint_step");
    return PIC_OK;
}

int pic_adjoint_step(pic_ctx* ctx, double* lam_fields, double* const* lam_x, double* const* lam_w,
                     double* lam_bext, void* stream)
{
    return adjoint_step_common(ctx, nullptr, 0, true, lam_fields, lam_x, lam_w, lam_bext, stream);
}

int pic_adjoint_record_bytes(const pic_ctx* ctx, size_t* bytes)
{
    if (!ctx || !bytes) return fail(nullptr, PIC_EINVAL, "null argument");
    *bytes = adjoint_record_bytes(ctx->c);
    return PIC_OK;
}

int pic_adjoint_record(pic_ctx* ctx, void* record, size_t bytes, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    if (!record) return fail(&c, PIC_EINVAL, "null record");
    const int r = adjoint_ready(c);
    if (r != PIC_OK) return r;
    if (bytes < adjoint_record_bytes(c)) return fail(&c, PIC_ESIZE, "record smaller than pic_adjoint_record_bytes");
    hipError_t e = launch_adjoint_record(c, record, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(&c, e, "adjoint_record");
    return PIC_OK;
}

int pic_adjoint_step_record(pic_ctx* ctx, const void* record, size_t bytes, double* lam_fields,
                            double* const* lam_x, double* const* lam_w, double* lam_bext, void* stream)
{
    if (!record) return fail(ctx ? &ctx->c : nullptr, PIC_EINVAL, "null record");
    return adjoint_step_common(ctx, record, bytes, true, lam_fields, lam_x, lam_w, lam_bext, stream);
}

int pic_adjoint_step_record_ordered(pic_ctx* ctx, const void* record, size_t bytes, double* lam_fields,
                                    double* const* lam_x, double* const* lam_w, double* lam_bext, void* stream)
{
    if (!record) return fail(ctx ? &ctx->c : nullptr, PIC_EINVAL, "null record");
    return adjoint_step_common(ctx, record, bytes, false, lam_fields, lam_x, lam_w, lam_bext, stream);
}

int pic_adjoint_reorder(pic_ctx* ctx, const void* from, const void* to, size_t bytes,
                        const double* const* in_x, const double* const* in_w, double* const* out_x,
                        double* const* out_w, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    const int r = adjoint_ready(c);
    if (r != PIC_OK) return r;
    if (!in_x || !in_w || !out_x || !out_w) return fail(&c, PIC_EINVAL, "null particle adjoint array");
    for (int i = 0; i < c.nsp; ++i) {
        const Species& sp = c.sp[i];
        if (!sp.d.mobile || sp.n == 0) continue;
        if (!in_x[i] || !in_w[i] || !out_x[i] || !out_w[i])
            return fail(&c, PIC_EINVAL, "null particle adjoint of a mobile species");
        if (in_x[i] == out_x[i] || in_w[i] == out_w[i] || in_x[i] == out_w[i] || in_w[i] == out_x[i])
            return fail(&c, PIC_EINVAL, "reorder is out of place: input and output must differ");
    }
    if ((from || to) && bytes < adjoint_record_bytes(c))
        return fail(&c, PIC_ESIZE, "record smaller than pic_adjoint_record_bytes");
    hipError_t e = launch_adjoint_reorder(c, from, to, in_x, in_w, out_x, out_w, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(&c, e, "adjoint_reorder");
    return PIC_OK;
}

int pic_solve_poisson(pic_ctx* ctx, int neutralize, double tol, int64_t* iterations, double* residual,
                      void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    if (neutralize != 0 && neutralize != 1) return fail(&c, PIC_EINVAL, "neutralize must be 0 or 1");
    if (c.g.xbc != 0) return fail(&c, PIC_ESTATE, "the Poisson solve is periodic; this context has an open x boundary");
    if (!(tol > 0.0)) tol = 1e-13;
    hipStream_t s = (hipStream_t)stream;
    // the total charge density goes to the Gauss reference's buffer, which is
    // recaptured before the next step
    hipError_t e = launch_total_rho(c, c.r0, s);
    int64_t it = 0;
    double res = 0.0;
    const int64_t nmax = std::max(c.k.n[0], std::max(c.k.n[1], c.k.n[2]));
    if (e == hipSuccess) e = solve_poisson(c, c.r0, neutralize != 0, tol, 50 * nmax + 200, &it, &res, s);
    c.r0_valid = false;
    if (e != hipSuccess) return hip_fail(&c, e, "solve_poisson");
    if (iterations) *iterations = it;
    if (residual) *residual = res;
    if (res > tol) return fail(&c, PIC_ESTATE, "Poisson solve did not reach the tolerance");
    return PIC_OK;
}

int pic_set_vector_potential(pic_ctx* ctx, const double* A, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    if (!A) return fail(&c, PIC_EINVAL, "null vector potential");
    if (c.k.field_form != 1) return fail(&c, PIC_ESTATE, "the context carries B (field_form 0)");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(c.avec, A, 3 * (size_t)c.k.ncell * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_b_of_a(c, s);
    if (e != hipSuccess) return hip_fail(&c, e, "set_vector_potential");
    return PIC_OK;
}

int pic_get_vector_potential(pic_ctx* ctx, double* A, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    if (!A) return fail(&c, PIC_EINVAL, "null output");
    if (c.k.field_form != 1) return fail(&c, PIC_ESTATE, "the context carries B (field_form 0)");
    hipError_t e = hipMemcpyAsync(A, c.avec, 3 * (size_t)c.k.ncell * 8, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(&c, e, "get_vector_potential");
    return PIC_OK;
}

int pic_diagnostics(pic_ctx* ctx, pic_diag* out, void* stream)
{
    if (!ctx || !out) return fail(ctx ? &ctx->c : nullptr, PIC_EINVAL, "null argument");
    Ctx& c = ctx->c;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = ensure_r0(c, s);
    if (e == hipSuccess) e = launch_diag(c, out, s);
    if (e != hipSuccess) return hip_fail(&c, e, "diagnostics");
    return PIC_OK;
}

int pic_diagnostics_static(pic_ctx* ctx, pic_diag* out, void* stream)
{
    if (!ctx || !out) return fail(ctx ? &ctx->c : nullptr, PIC_EINVAL, "null argument");
    Ctx& c = ctx->c;
    const size_t need = static_scratch_doubles(c) * sizeof(double);
    if (need > kStaticScratchBytes) {
        char msg[200];
        snprintf(msg, sizeof msg,
                 "pic_diagnostics_static: %lld cells need %zu bytes of static scratch, the maximum is %zu "
                 "(about %zu cells); use pic_diagnostics",
                 (long long)c.k.ncell, need, kStaticScratchBytes,
                 (size_t)(kStaticScratchBytes / sizeof(double)) - diag_partials_doubles(c.nsp) - 32);
        return fail(&c, PIC_ESIZE, msg);
    }
    double* sc = nullptr;
    hipError_t e = static_scratch_address(&sc);
    if (e != hipSuccess) return hip_fail(&c, e, "diagnostics_static: scratch address");
    hipStream_t s = (hipStream_t)stream;
    double* rho_m = sc;
    double* part = sc + align_up((size_t)c.k.ncell, 32);
    if (!c.r0_valid) {
        e = launch_capture_r0(c, s, rho_m);
        if (e == hipSuccess) c.r0_valid = true;
    }
    if (e == hipSuccess) e = launch_diag(c, out, s, rho_m, part);
    if (e != hipSuccess) return hip_fail(&c, e, "diagnostics_static");
    return PIC_OK;
}

int64_t pic_particle_count(const pic_ctx* ctx, int species)
{
    if (!ctx || species < 0 || species >= ctx->c.nsp) return -1;
    return ctx->c.sp[species].n;
}

int pic_get_particles(pic_ctx* ctx, int species, double* x, double* w, double* weight,
                      int64_t* id, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    if (species < 0 || species >= c.nsp || !c.sp[species].d.mobile)
        return fail(&c, PIC_EINVAL, "bad species index (or immobile species)");
    hipError_t e = launch_get(c, c.sp[species], x, w, weight, id, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(&c, e, "get_particles");
    return PIC_OK;
}

int pic_sort(pic_ctx* ctx, void* stream)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "null context");
    Ctx& c = ctx->c;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < c.nsp; ++i)
        if (c.sp[i].d.mobile) {
            hipError_t e = launch_sort(c, c.sp[i], s);
            if (e != hipSuccess) return hip_fail(&c, e, "sort");
        }
    c.since_sort = 0;
    return PIC_OK;
}

double pic_last_fallback_fraction(pic_ctx* ctx, void* stream)
{
    if (!ctx) return -1.0;
    Ctx& c = ctx->c;
    unsigned long long h[2] = {0, 0};
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(h, c.counters + 1, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess) return -1.0;
    if (hipStreamSynchronize(s) != hipSuccess) return -1.0;
    if (h[1] == 0) return -1.0;
    return (double)h[0] / (double)h[1];
}

double pic_last_migrant_fraction(pic_ctx* ctx, void* stream)
{
    if (!ctx) return -1.0;
    Ctx& c = ctx->c;
    unsigned long long h[3] = {0, 0, 0};
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(h, c.counters + 1, sizeof h, hipMemcpyDeviceToHost, s) != hipSuccess) return -1.0;
    if (hipStreamSynchronize(s) != hipSuccess) return -1.0;
    if (h[1] == 0) return -1.0;
    return (double)h[2] / (double)h[1];
}

int pic_timing_start(pic_ctx* ctx, int max_steps)
{
    if (!ctx || max_steps < 0) return fail(ctx ? &ctx->c : nullptr, PIC_EINVAL, "bad timing request");
    const size_t need = 5 * (size_t)max_steps;
    while (ctx->ev.size() < need) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return hip_fail(&ctx->c, r, "timing");
        ctx->ev.push_back(e);
    }
    ctx->timing_cap = max_steps;
    ctx->timing_used = 0;
    return PIC_OK;
}

int pic_timing_stop(pic_ctx* ctx, double ms[4], int64_t* steps)
{
    if (!ctx || !ms || !steps) return fail(ctx ? &ctx->c : nullptr, PIC_EINVAL, "null argument");
    for (int k = 0; k < 4; ++k) ms[k] = 0.0;
    const int n = ctx->timing_used;
    if (n > 0) {
        hipError_t r = hipEventSynchronize(ctx->ev[5 * (size_t)(n - 1) + 4]);
        if (r != hipSuccess) return hip_fail(&ctx->c, r, "timing");
        for (int st = 0; st < n; ++st)
            for (int k = 0; k < 4; ++k) {
                float t = 0.0f;
                r = hipEventElapsedTime(&t, ctx->ev[5 * (size_t)st + k], ctx->ev[5 * (size_t)st + k + 1]);
                if (r != hipSuccess) return hip_fail(&ctx->c, r, "timing");
                ms[k] += t;
            }
    }
    *steps = n;
    ctx->timing_cap = 0;
    ctx->timing_used = 0;
    return PIC_OK;
}

int pic_get_host_state(const pic_ctx* ctx, pic_host_state* out)
{
    if (!ctx || !out) return fail(nullptr, PIC_EINVAL, "null argument");
    const Ctx& c = ctx->c;
    *out = pic_host_state{};
    out->step = c.step;
    out->since_sort = c.since_sort;
    out->r0_valid = c.r0_valid ? 1 : 0;
    out->nsp = c.nsp;
    for (int i = 0; i < c.nsp; ++i) {
        out->n[i] = c.sp[i].n;
        out->sorted[i] = c.sp[i].sorted ? 1 : 0;
        out->copy[i] = c.sp[i].swapped;
    }
    return PIC_OK;
}

int pic_set_host_state(pic_ctx* ctx, const pic_host_state* in)
{
    if (!ctx || !in) return fail(ctx ? &ctx->c : nullptr, PIC_EINVAL, "null argument");
    Ctx& c = ctx->c;
    if (in->nsp != c.nsp || in->step < 0 || in->since_sort < 0)
        return fail(&c, PIC_ESTATE, "host state does not match this context");
    for (int i = 0; i < c.nsp; ++i)
        if (in->n[i] < 0 || (c.sp[i].d.mobile && in->n[i] > c.sp[i].d.capacity))
            return fail(&c, PIC_ESTATE, "host state particle count exceeds a capacity");
    c.step = in->step;
    c.since_sort = in->since_sort;
    c.r0_valid = in->r0_valid != 0;
    for (int i = 0; i < c.nsp; ++i) {
        Species& sp = c.sp[i];
        sp.n = sp.d.mobile ? in->n[i] : 0;
        sp.sorted = in->sorted[i] != 0;
        if (sp.d.mobile && (in->copy[i] & 1) != sp.swapped) {
            const PartArrays t = sp.cur;
            sp.cur = sp.alt;
            sp.alt = t;
            sp.swapped ^= 1;
        }
    }
    return PIC_OK;
}

void pic_destroy(pic_ctx* ctx) { delete ctx; }

}  // extern "C"
