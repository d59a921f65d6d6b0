// C ABI of the LEE lattice Boltzmann library: argument checks, coefficient setup, dispatch.
// The step launch sequences live in step_<set>.hip (one translation unit per velocity set).
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>

#include "internal.hpp"

using namespace lbm::api;

namespace lbm {
namespace api {

namespace {
thread_local std::string g_err;
}

lbm_status fail(lbm_status st, const char *fmt, ...) {
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    g_err = msg;
    return st;
}

lbm_status ok() {
    g_err.clear();
    return LBM_OK;
}

}  // namespace api
}  // namespace lbm

namespace {

lbm_status launch_init(lbm_lee *h, const double *rho, const double *u, const double *theta, hipStream_t st) {
    return visit(h->desc.lattice, h->desc.storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        using ST = decltype(sto);
        auto k = field_coef<VS::Q>(h);
        auto *dst = static_cast<typename ST::elem *>(h->buf[h->cur]);
        auto *other = static_cast<typename ST::elem *>(rest_copy_buffer(h));
        init_equilibrium<VS, ST><<<blocks_for(h->N), 256, 0, st>>>(rho, u, theta, dst, other, h->N, k, layout_fresh(h));
        return launch_check();
    });
}

// Equilibrium of fields given on a sub-box (n_sub cells at origin), the state at rest elsewhere;
// n_sub = {0, 0, 0} sets the whole box at rest (the field pointers are then not read).
lbm_status launch_init_region(lbm_lee *h, const int64_t origin[3], const int64_t n_sub[3], const double *rho,
                              const double *u, const double *theta, hipStream_t st) {
    return visit(h->desc.lattice, h->desc.storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        using ST = decltype(sto);
        auto k = field_coef<VS::Q>(h);
        auto *dst = static_cast<typename ST::elem *>(h->buf[h->cur]);
        auto *other = static_cast<typename ST::elem *>(rest_copy_buffer(h));
        init_region<VS, ST><<<blocks_for(h->N), 256, 0, st>>>(rho, u, theta, dst, other, h->nx, h->ny, h->N,
                                                              (int)origin[0], (int)origin[1], (int)origin[2],
                                                              (int)n_sub[0], (int)n_sub[1], (int)n_sub[2], k,
                                                              layout_fresh(h));
        return launch_check();
    });
}

lbm_status choose_scale(lbm_lee *h, const double *rho, const double *u, const double *theta, hipStream_t st) {
    if (!is_scaled(h->desc.storage)) {
        h->S = 1.0;
        return LBM_OK;
    }
    if (h->desc.store_scale > 0.0) {
        h->S = h->desc.store_scale;
        return LBM_OK;
    }
    double *part = static_cast<double *>(h->scratch);
    double *res = part + 6 * kReduceBlocks;
    lbm_status s = visit(h->desc.lattice, LBM_F64, [&](auto vs, auto) -> lbm_status {
        using VS = decltype(vs);
        auto k = field_coef<VS::Q>(h);  // scale-independent parts only are used
        scale_partials<VS><<<kReduceBlocks, 256, 0, st>>>(rho, u, theta, h->N, k, part);
        return launch_check();
    });
    if (s != LBM_OK) return s;
    reduce_partials<1><<<1, 256, 0, st>>>(part, kReduceBlocks, res, 1u);
    if ((s = launch_check()) != LBM_OK) return s;
    double mx = 0.0;
    LBM_HIP(hipMemcpyAsync(&mx, res, sizeof(double), hipMemcpyDeviceToHost, st));
    LBM_HIP(hipStreamSynchronize(st));
    if (!(mx > 0.0) || !std::isfinite(mx)) {
        h->S = 1.0;
    } else {
        int ex;
        std::frexp(mx, &ex);  // mx = m 2^ex, m in [1/2, 1)
        // S mx in [1/2, 1) for the floating formats, in [2^13, 2^14) for fixed point
        h->S = std::ldexp(1.0, (h->desc.storage == LBM_I16 ? 14 : 0) - ex);
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

const char *lbm_lee_last_error(void) { return g_err.c_str(); }

const char *lbm_lee_version(void) { return "lbm_lee 0.1 gfx950"; }

lbm_status lbm_lee_lattice_info(int32_t lattice, lbm_lattice_info *out) {
    if (!out) return fail(LBM_E_INVALID, "out is NULL");
    LatticeTable t;
    if (!build_lattice(lattice, &t)) return fail(LBM_E_INVALID, "unknown lattice id %d", lattice);
    std::memset(out, 0, sizeof(*out));
    out->D = t.D;
    out->Q = t.Q;
    for (int i = 0; i < t.Q; ++i) {
        for (int a = 0; a < 3; ++a) out->c[i][a] = t.c[i][a];
        out->fstar[i] = t.f[i];
        out->beta[i] = t.beta[i];
    }
    out->rho0 = t.rho0;
    out->theta0 = t.theta0;
    out->gamma = t.gamma;
    out->a1 = t.a1;
    out->a2 = t.a2;
    out->b = t.b;
    out->c1 = t.c1;
    out->c2 = t.c2;
    std::snprintf(out->name, sizeof out->name, "%s", t.name);
    return ok();
}

lbm_status lbm_lee_dimensional_scaling(int32_t lattice, double rho0_dim, double theta0_dim, double x_star,
                                       lbm_lee_scaling *out) {
    if (!out) return fail(LBM_E_INVALID, "out is NULL");
    LatticeTable t;
    if (!build_lattice(lattice, &t)) return fail(LBM_E_INVALID, "unknown lattice id %d", lattice);
    if (!(rho0_dim > 0.0) || !(theta0_dim > 0.0) || !(x_star > 0.0) || !std::isfinite(rho0_dim) ||
        !std::isfinite(theta0_dim) || !std::isfinite(x_star))
        return fail(LBM_E_INVALID, "rho0_dim, theta0_dim and x_star must be finite and > 0");
    out->rho_star = rho0_dim / t.rho0;
    out->theta_star = theta0_dim / t.theta0;
    out->u_star = std::sqrt(out->theta_star);
    out->x_star = x_star;
    out->t_star = x_star / out->u_star;
    return ok();
}

lbm_status lbm_lee_dimensional_steps(const lbm_lee_scaling *s, double t_dim, double dt, int64_t *nsteps,
                                     double *t_end, double *offset) {
    if (!s) return fail(LBM_E_INVALID, "scaling is NULL");
    if (!(s->t_star > 0.0) || !std::isfinite(s->t_star)) return fail(LBM_E_INVALID, "scaling has no valid t_star");
    if (!(t_dim >= 0.0) || !std::isfinite(t_dim)) return fail(LBM_E_INVALID, "t_dim must be finite and >= 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(LBM_E_INVALID, "dt must be finite and > 0");
    const double T = t_dim / s->t_star;
    const double n = std::round(T / dt);
    if (!(n <= 4.6e18)) return fail(LBM_E_INVALID, "more than 2^62 steps");
    if (nsteps) *nsteps = (int64_t)n;
    if (t_end) *t_end = n * dt;
    if (offset) *offset = T - n * dt;
    return ok();
}

size_t lbm_lee_state_bytes(const lbm_lee_desc *d) {
    LatticeTable t;
    if (check_desc(d, &t) != LBM_OK) return 0;
    return (size_t)t.Q * (size_t)(d->n[0] * d->n[1] * d->n[2]) * elem_size(d->storage);
}

size_t lbm_lee_scratch_bytes(const lbm_lee_desc *d) {
    LatticeTable t;
    if (check_desc(d, &t) != LBM_OK) return 0;
    return kScratchBytes;
}

lbm_status lbm_lee_collision_constants(const lbm_lee_desc *desc, double H[16], double WB[16], double *keep) {
    if (!H || !WB || !keep) return fail(LBM_E_INVALID, "H, WB or keep is NULL");
    LatticeTable t;
    const lbm_status s = check_desc(desc, &t);
    if (s != LBM_OK) return s;
    double h2[kShells][kShells], w2[kShells][kShells];
    fold_constants(t, desc->storage, desc->store_scale > 0.0 ? desc->store_scale : 1.0, desc->tau, 1.0, h2, w2, *keep);
    for (int to = 0; to < kShells; ++to)
        for (int from = 0; from < kShells; ++from) {
            H[to * kShells + from] = h2[to][from];
            WB[to * kShells + from] = w2[to][from];
        }
    return ok();
}

double lbm_lee_bytes_per_update(const lbm_lee_desc *d) {
    LatticeTable t;
    if (check_desc(d, &t) != LBM_OK) return 0.0;
    const int moved = skip_rest(t, d) ? t.Q - 1 : t.Q;
    return 2.0 * moved * (double)elem_size(d->storage);
}

lbm_status lbm_lee_init(const lbm_lee_desc *desc, void *pop_a, void *pop_b, size_t bytes_each, const double *rho,
                        const double *u, const double *theta, void *scratch, size_t scratch_bytes, void *stream,
                        lbm_lee_handle *out) {
    if (!out) return fail(LBM_E_INVALID, "out is NULL");
    *out = nullptr;
    LatticeTable tab;
    lbm_status s = check_desc(desc, &tab);
    if (s != LBM_OK) return s;
    const size_t N = (size_t)(desc->n[0] * desc->n[1] * desc->n[2]);
    const size_t need = (size_t)tab.Q * N * elem_size(desc->storage);
    const bool inplace = (desc->tune & kTuneInPlace) != 0;
    if (inplace) {
        if (!pop_a) return fail(LBM_E_INVALID, "pop_a must not be NULL");
        if (!aligned256(pop_a)) return fail(LBM_E_INVALID, "the population buffer must be 256-byte aligned");
        if (bytes_each < need) return fail(LBM_E_INVALID, "the population buffer holds %zu bytes, need %zu", bytes_each, need);
        pop_b = nullptr;  // one buffer
    } else {
        if (!pop_a || !pop_b || pop_a == pop_b) return fail(LBM_E_INVALID, "pop_a and pop_b must be two distinct buffers");
        if (!aligned256(pop_a) || !aligned256(pop_b)) return fail(LBM_E_INVALID, "population buffers must be 256-byte aligned");
        if (bytes_each < need) return fail(LBM_E_INVALID, "population buffers hold %zu bytes, need %zu", bytes_each, need);
        const char *a = static_cast<const char *>(pop_a), *b = static_cast<const char *>(pop_b);
        if (a < b + need && b < a + need) return fail(LBM_E_INVALID, "population buffers overlap");
    }
    const bool at_rest = !rho && !u && !theta;
    if (!at_rest && (!rho || !u || !theta))
        return fail(LBM_E_INVALID, "initial fields must be all given or all NULL (the state at rest)");
    if (!scratch || !aligned256(scratch) || scratch_bytes < kScratchBytes)
        return fail(LBM_E_INVALID, "scratch must be 256-byte aligned and hold >= %zu bytes", kScratchBytes);
    lbm_lee *h = new (std::nothrow) lbm_lee;
    if (!h) return fail(LBM_E_INVALID, "out of host memory");
    h->desc = *desc;
    h->tab = tab;
    h->N = N;
    h->nx = (int)desc->n[0];
    h->ny = (int)desc->n[1];
    h->nz = (int)desc->n[2];
    h->buf[0] = pop_a;
    h->buf[1] = pop_b;
    h->cur = 0;
    h->steps = 0;
    h->scratch = scratch;
    h->scratch_bytes = scratch_bytes;
    h->S = 1.0;
    h->cus = 0;
    h->net = nullptr;
    h->ghost = nullptr;
    h->skip0 = skip_rest(tab, desc);
    h->inplace = inplace;
    h->phase = 0;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            h->cus = 0;  // persistent launches then fall back to the full grid
        (void)hipGetLastError();
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (at_rest) {
        const int64_t zero[3] = {0, 0, 0};
        h->S = (is_scaled(desc->storage) && desc->store_scale > 0.0) ? desc->store_scale : 1.0;
        s = launch_init_region(h, zero, zero, nullptr, nullptr, nullptr, st);
    } else if ((s = choose_scale(h, rho, u, theta, st)) == LBM_OK) {
        s = launch_init(h, rho, u, theta, st);
    }
    if (s != LBM_OK) {
        delete h;
        return s;
    }
    *out = h;
    return ok();
}

lbm_status lbm_lee_reinit(lbm_lee_handle h, const double *rho, const double *u, const double *theta, void *stream) {
    if (!h) return fail(LBM_E_INVALID, "handle is NULL");
    if (!rho || !u || !theta) return fail(LBM_E_INVALID, "initial fields must not be NULL");
    h->cur = 0;
    h->steps = 0;
    h->hist_valid = false;
    h->phase = 0;
    lbm_status s = launch_init(h, rho, u, theta, static_cast<hipStream_t>(stream));
    return s == LBM_OK ? ok() : s;
}

namespace {
lbm_status check_region(const lbm_lee *h, const int64_t origin[3], const int64_t n_sub[3]) {
    if (!origin || !n_sub) return fail(LBM_E_INVALID, "origin and n_sub must not be NULL");
    for (int a = 0; a < 3; ++a)
        if (n_sub[a] < 1 || origin[a] < 0 || origin[a] + n_sub[a] > h->desc.n[a])
            return fail(LBM_E_INVALID, "sub-box (axis %d) must lie inside the box", a);
    return LBM_OK;
}
}  // namespace

lbm_status lbm_lee_reinit_region(lbm_lee_handle h, const int64_t origin[3], const int64_t n_sub[3], const double *rho,
                                 const double *u, const double *theta, void *stream) {
    if (!h) return fail(LBM_E_INVALID, "handle is NULL");
    if (!rho || !u || !theta) return fail(LBM_E_INVALID, "fields must not be NULL");
    lbm_status s = check_region(h, origin, n_sub);
    if (s != LBM_OK) return s;
    h->cur = 0;
    h->steps = 0;
    h->hist_valid = false;
    h->phase = 0;
    s = launch_init_region(h, origin, n_sub, rho, u, theta, static_cast<hipStream_t>(stream));
    return s == LBM_OK ? ok() : s;
}

lbm_status lbm_lee_moments_region(lbm_lee_handle h, const int64_t origin[3], const int64_t n_sub[3], void *p, void *u,
                                  void *rho, void *theta, int32_t out_is_f64, void *stream) {
    if (!h) return fail(LBM_E_INVALID, "handle is NULL");
    lbm_status s = check_region(h, origin, n_sub);
    if (s != LBM_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t Ns = (size_t)(n_sub[0] * n_sub[1] * n_sub[2]);
    s = visit(h->desc.lattice, h->desc.storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        using ST = decltype(sto);
        auto k = field_coef<VS::Q>(h);
        const auto *src = static_cast<const typename ST::elem *>(h->buf[h->cur]);
        const int o0 = (int)origin[0], o1 = (int)origin[1], o2 = (int)origin[2];
        const int s0 = (int)n_sub[0], s1 = (int)n_sub[1], s2 = (int)n_sub[2];
        if (out_is_f64)
            moments_region_kernel<VS, ST, double><<<blocks_for(Ns), 256, 0, st>>>(
                src, h->N, h->nx, h->ny, o0, o1, o2, s0, s1, s2, k, (double *)p, (double *)u, (double *)rho,
                (double *)theta, layout_now(h));
        else
            moments_region_kernel<VS, ST, float><<<blocks_for(Ns), 256, 0, st>>>(
                src, h->N, h->nx, h->ny, o0, o1, o2, s0, s1, s2, k, (float *)p, (float *)u, (float *)rho,
                (float *)theta, layout_now(h));
        return launch_check();
    });
    return s == LBM_OK ? ok() : s;
}

lbm_status lbm_lee_step(lbm_lee_handle h, int64_t nsteps, void *stream) {
    if (!h) return fail(LBM_E_INVALID, "handle is NULL");
    if (nsteps < 0) return fail(LBM_E_INVALID, "nsteps must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (h->desc.bc == LBM_BC_MLP && (!h->net || !h->ghost))
        return fail(LBM_E_STATE, "an LBM_BC_MLP handle needs lbm_lee_set_closure before stepping");
    lbm_status s;
    switch (h->desc.lattice) {
        case LBM_D1Q3: s = step_lattice<VS_D1Q3>(h, nsteps, st); break;
        case LBM_D2Q5:
        case LBM_D2Q5_DIA: s = step_lattice<VS_D2Q5>(h, nsteps, st); break;
        case LBM_D2Q9: s = step_lattice<VS_D2Q9>(h, nsteps, st); break;
        case LBM_D3Q7:
        case LBM_D3Q7_DIA: s = step_lattice<VS_D3Q7>(h, nsteps, st); break;
        case LBM_D3Q9: s = step_lattice<VS_D3Q9>(h, nsteps, st); break;
        case LBM_D3Q13: s = step_lattice<VS_D3Q13>(h, nsteps, st); break;
        case LBM_D3Q19: s = step_lattice<VS_D3Q19>(h, nsteps, st); break;
        case LBM_D3Q27: s = step_lattice<VS_D3Q27>(h, nsteps, st); break;
        default: s = fail(LBM_E_INVALID, "unknown lattice id %d", h->desc.lattice);
    }
    return s == LBM_OK ? ok() : s;
}

lbm_status lbm_lee_moments(lbm_lee_handle h, void *p, void *u, void *rho, void *theta, int32_t out_is_f64,
                           void *stream) {
    if (!h) return fail(LBM_E_INVALID, "handle is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    lbm_status s = visit(h->desc.lattice, h->desc.storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        using ST = decltype(sto);
        auto k = field_coef<VS::Q>(h);
        const auto *src = static_cast<const typename ST::elem *>(h->buf[h->cur]);
        if (out_is_f64)
            moments_kernel<VS, ST, double><<<blocks_for(h->N), 256, 0, st>>>(
                src, h->N, k, (double *)p, (double *)u, (double *)rho, (double *)theta, layout_now(h));
        else
            moments_kernel<VS, ST, float><<<blocks_for(h->N), 256, 0, st>>>(
                src, h->N, k, (float *)p, (float *)u, (float *)rho, (float *)theta, layout_now(h));
        return launch_check();
    });
    return s == LBM_OK ? ok() : s;
}

lbm_status lbm_lee_l2_energy(lbm_lee_handle h, double out[2], void *stream) {
    if (!h || !out) return fail(LBM_E_INVALID, "handle or out is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(h->scratch);
    double *res = part + 6 * kReduceBlocks;
    lbm_status s = visit(h->desc.lattice, h->desc.storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        using ST = decltype(sto);
        auto k = field_coef<VS::Q>(h);
        const auto *src = static_cast<const typename ST::elem *>(h->buf[h->cur]);
        energy_partials<VS, ST><<<kReduceBlocks, 256, 0, st>>>(src, h->N, k, part);
        return launch_check();
    });
    if (s != LBM_OK) return s;
    reduce_partials<2><<<1, 256, 0, st>>>(part, kReduceBlocks, res, 0u);
    if ((s = launch_check()) != LBM_OK) return s;
    LBM_HIP(hipMemcpyAsync(out, res, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    LBM_HIP(hipStreamSynchronize(st));
    return ok();
}

lbm_status lbm_lee_error_norms(lbm_lee_handle h, const double *ref_p, const double *ref_u, double out[6],
                               void *stream) {
    if (!h || !out || !ref_p) return fail(LBM_E_INVALID, "handle, ref_p or out is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *part = static_cast<double *>(h->scratch);
    double *res = part + 6 * kReduceBlocks;
    lbm_status s = visit(h->desc.lattice, h->desc.storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        using ST = decltype(sto);
        auto k = field_coef<VS::Q>(h);
        const auto *src = static_cast<const typename ST::elem *>(h->buf[h->cur]);
        error_partials<VS, ST><<<kReduceBlocks, 256, 0, st>>>(src, h->N, k, ref_p, ref_u, part, layout_now(h));
        return launch_check();
    });
    if (s != LBM_OK) return s;
    reduce_partials<6><<<1, 256, 0, st>>>(part, kReduceBlocks, res, (1u << 2) | (1u << 5));
    if ((s = launch_check()) != LBM_OK) return s;
    LBM_HIP(hipMemcpyAsync(out, res, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
    LBM_HIP(hipStreamSynchronize(st));
    return ok();
}

lbm_status lbm_lee_export_f64(lbm_lee_handle h, double *g, void *stream) {
    if (!h || !g) return fail(LBM_E_INVALID, "handle or g is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    lbm_status s = visit(h->desc.lattice, h->desc.storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        using ST = decltype(sto);
        auto k = field_coef<VS::Q>(h);
        const auto *src = static_cast<const typename ST::elem *>(h->buf[h->cur]);
        export_f64<VS, ST><<<blocks_for((size_t)VS::Q * h->N), 256, 0, st>>>(src, h->N, k, g, layout_now(h));
        return launch_check();
    });
    return s == LBM_OK ? ok() : s;
}

lbm_status lbm_lee_import_f64(lbm_lee_handle h, const double *g, int64_t steps_done, void *stream) {
    if (!h || !g) return fail(LBM_E_INVALID, "handle or g is NULL");
    if (steps_done < 0) return fail(LBM_E_INVALID, "steps_done must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    lbm_status s = visit(h->desc.lattice, h->desc.storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        using ST = decltype(sto);
        auto k = field_coef<VS::Q>(h);
        auto *dst = static_cast<typename ST::elem *>(h->buf[h->cur]);
        auto *other = static_cast<typename ST::elem *>(rest_copy_buffer(h));
        import_f64<VS, ST><<<blocks_for((size_t)VS::Q * h->N), 256, 0, st>>>(g, h->N, k, dst, other, layout_fresh(h));
        return launch_check();
    });
    if (s != LBM_OK) return s;
    h->steps = steps_done;
    h->hist_valid = false;
    h->phase = 0;
    return ok();
}

lbm_status lbm_lee_current(lbm_lee_handle h, void **pop, int64_t *steps_done) {
    if (!h) return fail(LBM_E_INVALID, "handle is NULL");
    if (pop) *pop = h->buf[h->cur];
    if (steps_done) *steps_done = h->steps;
    return ok();
}

double lbm_lee_store_scale(lbm_lee_handle h) { return h ? h->S : 0.0; }

int32_t lbm_lee_resolved_variant(lbm_lee_handle h) { return h ? resolve_variant(h) : -1; }

void lbm_lee_destroy(lbm_lee_handle h) { delete h; }

size_t lbm_lee_ghost_bytes(const lbm_lee_desc *d) {
    LatticeTable t;
    if (check_desc(d, &t) != LBM_OK || d->bc != LBM_BC_MLP) return 0;
    // ghost values, then two history buffers of one strip per node (read one, write the other)
    return (size_t)face_node_count(t, d->n) * (size_t)(net_outputs(t) + 2 * 3 * t.Q) * sizeof(float);
}

lbm_status lbm_lee_set_closure(lbm_lee_handle h, const float *params, void *ghost, size_t ghost_bytes) {
    if (!h) return fail(LBM_E_INVALID, "handle is NULL");
    if (h->desc.bc != LBM_BC_MLP) return fail(LBM_E_STATE, "the handle's boundary is not LBM_BC_MLP");
    if (!params || !ghost) return fail(LBM_E_INVALID, "params and ghost must not be NULL");
    if (ghost_bytes < lbm_lee_ghost_bytes(&h->desc)) return fail(LBM_E_INVALID, "ghost buffer too small");
    if (reinterpret_cast<uintptr_t>(params) & 3 || reinterpret_cast<uintptr_t>(ghost) & 3)
        return fail(LBM_E_INVALID, "params and ghost must be 4-byte aligned");
    if (!h->aux) {
        hipStream_t a = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipStreamCreateWithFlags(&a, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&e0, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            if (a) (void)hipStreamDestroy(a);
            (void)hipGetLastError();
            return fail(LBM_E_HIP, "cannot create the closure's helper stream and events");
        }
        h->aux = a;
        h->fork = e0;
        h->join = e1;
    }
    h->net = params;
    h->ghost = static_cast<float *>(ghost);
    h->hist_valid = false;
    return ok();
}

lbm_status lbm_nrbc_dims(int32_t lattice, int32_t dims[4]) {
    LatticeTable t;
    if (!dims) return fail(LBM_E_INVALID, "dims is NULL");
    if (!build_lattice(lattice, &t)) return fail(LBM_E_INVALID, "unknown lattice id %d", lattice);
    if (!net_fits(t)) return fail(LBM_E_UNSUPPORTED, "the closure network takes sets of up to 21 velocities");
    dims[0] = (int32_t)net_inputs(t);
    dims[1] = net_outputs(t);
    dims[2] = kHidden;
    dims[3] = (int32_t)net_params(t);
    return ok();
}

int64_t lbm_nrbc_face_nodes(const lbm_lee_desc *d) {
    LatticeTable t;
    if (check_desc(d, &t) != LBM_OK) return -1;
    return face_node_count(t, d->n);
}

namespace {
constexpr int kNetGrid = 256;  // blocks of the gradient kernel: 1024 partial rows
}

size_t lbm_nrbc_workspace_bytes(int32_t lattice, int64_t count) {
    LatticeTable t;
    if (!build_lattice(lattice, &t) || count < 0) return 0;
    (void)count;
    return (size_t)kNetGrid * 4 * (size_t)(net_params(t) + 1) * sizeof(float) + 256;
}

lbm_status lbm_nrbc_forward(int32_t lattice, const float *params, const float *strips, int64_t count, float *out,
                            void *stream) {
    if (!params || !strips || !out || count < 0) return fail(LBM_E_INVALID, "bad arguments");
    if (count == 0) return ok();
    hipStream_t st = static_cast<hipStream_t>(stream);
    const long long tiles = (count + 15) / 16;
    const unsigned grid = (unsigned)std::min<long long>((tiles + 3) / 4, 4096);
    lbm_status s = visit(lattice, LBM_F32, [&](auto vs, auto) -> lbm_status {
        using VS = decltype(vs);
        if constexpr (NetGeom<VS>::fits) {
            nrbc_forward_kernel<VS><<<grid, 256, 0, st>>>(params, strips, count, out);
            return launch_check();
        }
        return fail(LBM_E_UNSUPPORTED, "the closure network takes sets of up to 21 velocities");
    });
    return s == LBM_OK ? ok() : s;
}

lbm_status lbm_nrbc_loss_grad(int32_t lattice, const float *params, const float *strips, const float *targets,
                              int64_t count, float *grad, float *loss, void *workspace, size_t workspace_bytes,
                              void *stream) {
    if (!params || !strips || !targets || !grad || !workspace || count <= 0)
        return fail(LBM_E_INVALID, "bad arguments");
    if (workspace_bytes < lbm_nrbc_workspace_bytes(lattice, count)) return fail(LBM_E_INVALID, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    lbm_status s = visit(lattice, LBM_F32, [&](auto vs, auto) -> lbm_status {
        using VS = decltype(vs);
        if constexpr (!NetGeom<VS>::fits) {
            return fail(LBM_E_UNSUPPORTED, "the closure network takes sets of up to 21 velocities");
        } else {
            using G = NetGeom<VS>;
            // layout: [counter (256 bytes)][kNetGrid * 4 partial rows]
            auto *nvalid = static_cast<unsigned long long *>(workspace);
            float *ws = reinterpret_cast<float *>(static_cast<char *>(workspace) + 256);
            nrbc_zero_counter<<<1, 1, 0, st>>>(nvalid);
            nrbc_count_valid<VS><<<blocks_for((size_t)count), 256, 0, st>>>(strips, count, nvalid);
            nrbc_grad_kernel<VS><<<kNetGrid, 256, 0, st>>>(params, strips, targets, count, nvalid, ws);
            lbm_status ls = launch_check();
            if (ls != LBM_OK) return ls;
            nrbc_reduce_kernel<<<(G::NPARAM + 1 + 255) / 256, 256, 0, st>>>(ws, kNetGrid * 4, G::NPARAM, nvalid, G::NOUT,
                                                                           grad, loss);
            return launch_check();
        }
    });
    return s == LBM_OK ? ok() : s;
}

lbm_status lbm_nrbc_adam(int64_t n, float *params, const float *grad, float *m, float *v, int64_t t, float lr,
                         float beta1, float beta2, float eps, void *stream) {
    if (!params || !grad || !m || !v || n <= 0 || t < 1) return fail(LBM_E_INVALID, "bad arguments");
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
    nrbc_adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, static_cast<hipStream_t>(stream)>>>(
        n, params, grad, m, v, lr, beta1, beta2, eps, c1, c2);
    lbm_status s = launch_check();
    return s == LBM_OK ? ok() : s;
}

lbm_status lbm_nrbc_gather(lbm_lee_handle outer, const int64_t origin[3], const lbm_lee_desc *inner,
                           const int64_t *node_ids, int64_t count, float *strips, int64_t strip_stride, float *targets,
                           void *stream) {
    if (!outer || !origin || !inner || !node_ids || !strips || count < 0) return fail(LBM_E_INVALID, "bad arguments");
    LatticeTable t;
    lbm_status s = check_desc(inner, &t);
    if (s != LBM_OK) return s;
    if (strip_stride < 3 * t.Q) return fail(LBM_E_INVALID, "strip_stride must be >= 3 Q = %d", 3 * t.Q);
    if (inner->lattice != outer->desc.lattice) return fail(LBM_E_INVALID, "inner and outer lattices differ");
    const int spare = targets ? 1 : 0;  // targets read one cell beyond the inner box
    for (int a = 0; a < t.D; ++a)
        if (origin[a] < spare || origin[a] + inner->n[a] + spare > outer->desc.n[a] || inner->n[a] < 3)
            return fail(LBM_E_INVALID, "inner box (axis %d) must sit inside the outer box%s", a,
                        targets ? " with one cell to spare" : "");
    if (count == 0) return ok();
    hipStream_t st = static_cast<hipStream_t>(stream);
    s = visit(outer->desc.lattice, outer->desc.storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        using ST = decltype(sto);
        const auto ft = face_table<VS>(t, inner->n);
        const auto fk = field_coef<VS::Q>(outer);
        const auto *src = static_cast<const typename ST::elem *>(outer->buf[outer->cur]);
        gather_pairs_kernel<VS, ST><<<blocks_for((size_t)count), 256, 0, st>>>(
            src, outer->N, outer->nx, outer->ny, (int)origin[0], (int)(t.D > 1 ? origin[1] : 0),
            (int)(t.D > 2 ? origin[2] : 0), reinterpret_cast<const long long *>(node_ids), count, strips,
            (long long)strip_stride, targets, ft, fk);
        return launch_check();
    });
    return s == LBM_OK ? ok() : s;
}

namespace {
// Deterministic two-pass comparison of box a with its place in box b on `scratch` (partials of
// the kReduceBlocks blocks, then the three results); the caller has checked the arguments.
lbm_status compare_fields_on(const double *a, const int64_t n_a[3], const double *b, const int64_t n_b[3],
                             const int64_t origin[3], double out[3], void *scratch, hipStream_t st) {
    double *part = static_cast<double *>(scratch);
    double *res = part + 6 * kReduceBlocks;
    compare_partials<<<kReduceBlocks, 256, 0, st>>>(a, (int)n_a[0], (int)n_a[1], (int)n_a[2], b, (int)n_b[0],
                                                    (int)n_b[1], (int)origin[0], (int)origin[1], (int)origin[2], part);
    lbm_status s = launch_check();
    if (s != LBM_OK) return s;
    reduce_partials<3><<<1, 256, 0, st>>>(part, kReduceBlocks, res, 1u << 2);
    if ((s = launch_check()) != LBM_OK) return s;
    LBM_HIP(hipMemcpyAsync(out, res, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    LBM_HIP(hipStreamSynchronize(st));
    return LBM_OK;
}

lbm_status check_compare_args(const double *a, const int64_t n_a[3], const double *b, const int64_t n_b[3],
                              const int64_t origin[3], double out[3]) {
    if (!a || !n_a || !b || !n_b || !origin || !out) return fail(LBM_E_INVALID, "bad arguments");
    for (int d = 0; d < 3; ++d)
        if (n_a[d] < 1 || origin[d] < 0 || origin[d] + n_a[d] > n_b[d] || n_a[d] > (1 << 30) || n_b[d] > (1 << 30))
            return fail(LBM_E_INVALID, "box a must lie inside box b (axis %d)", d);
    return LBM_OK;
}

// Scratch of lbm_lee_compare_fields_static: a file-scope device array, so that entry point
// needs no allocation and no workspace argument.  Every GPU the library runs on holds its own
// copy until the process ends.  In host code the array's name is only a stand-in for the
// symbol: its device address, different on each GPU, comes from hipGetSymbolAddress, taken once
// per device (with that device current) on the entry point's first call there and kept below.
constexpr size_t kStaticScratchBytes = kScratchBytes;  // 96 KiB: kReduceBlocks partial rows + results
static_assert((size_t)(6 * kReduceBlocks + 6) * sizeof(double) <= kStaticScratchBytes, "reduction layout");
static __device__ __align__(256) unsigned char static_scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_scratch_mu;
void *g_static_scratch_ptr[kMaxDevices] = {};

lbm_status static_scratch_on_current_device(void **out) {
    int dev = -1;
    LBM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_static_scratch_mu);
    if (!g_static_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(static_scratch));
        if (e != hipSuccess || !p)
            return fail(LBM_E_HIP, "hipGetSymbolAddress(static_scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_static_scratch_ptr[dev] = p;
    }
    *out = g_static_scratch_ptr[dev];
    return LBM_OK;
}
}  // namespace

lbm_status lbm_lee_compare_fields(const double *a, const int64_t n_a[3], const double *b, const int64_t n_b[3],
                                  const int64_t origin[3], double out[3], void *scratch, size_t scratch_bytes,
                                  void *stream) {
    lbm_status s = check_compare_args(a, n_a, b, n_b, origin, out);
    if (s != LBM_OK) return s;
    if (!scratch || scratch_bytes < kScratchBytes || !aligned256(scratch))
        return fail(LBM_E_INVALID, "scratch too small or misaligned");
    s = compare_fields_on(a, n_a, b, n_b, origin, out, scratch, static_cast<hipStream_t>(stream));
    return s == LBM_OK ? ok() : s;
}

lbm_status lbm_lee_compare_fields_static(const double *a, const int64_t n_a[3], const double *b,
                                         const int64_t n_b[3], const int64_t origin[3], double out[3], void *stream) {
    lbm_status s = check_compare_args(a, n_a, b, n_b, origin, out);
    if (s != LBM_OK) return s;
    void *scratch = nullptr;
    if ((s = static_scratch_on_current_device(&scratch)) != LBM_OK) return s;
    s = compare_fields_on(a, n_a, b, n_b, origin, out, scratch, static_cast<hipStream_t>(stream));
    return s == LBM_OK ? ok() : s;
}

lbm_status lbm_lee_device_copy(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src) return fail(LBM_E_INVALID, "NULL pointer");
    if (bytes % 16 || (reinterpret_cast<uintptr_t>(dst) & 15) || (reinterpret_cast<uintptr_t>(src) & 15))
        return fail(LBM_E_INVALID, "copy needs 16-byte aligned pointers and a size multiple of 16");
    const size_t n16 = bytes / 16;
    if (n16 == 0) return ok();
    const size_t want = (n16 + 255) / 256;
    const unsigned blocks = (unsigned)(want < 65536 ? want : 65536);
    copy16<<<blocks, 256, 0, static_cast<hipStream_t>(stream)>>>(static_cast<const f32x4 *>(src),
                                                                   static_cast<f32x4 *>(dst), n16);
    lbm_status s = launch_check();
    return s == LBM_OK ? ok() : s;
}

}  // extern "C"
