// C ABI of the LEE lattice Boltzmann library: argument checks, coefficient setup, dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/lbm_lee.h"
#include "kernels.hpp"
#include "nrbc.hpp"
#include "open_bc.hpp"
#include "temporal.hpp"
#include "tables.hpp"

using namespace lbm;

struct lbm_lee {
    lbm_lee_desc desc;
    LatticeTable tab;
    size_t N;
    int nx, ny, nz;
    void *buf[2];
    int cur;
    int64_t steps;
    void *scratch;
    size_t scratch_bytes;
    double S;  // storage scale (1 for F64/F32)
    int cus;   // compute units of the device (persistent launches)
    const float *net;  // LBM_BC_MLP: closure parameters (caller-owned)
    float *ghost;      // LBM_BC_MLP: ghost buffer (caller-owned)
    bool skip0;        // rest population left out of the step (invariant under it)
    bool inplace = false;  // LBM_TUNE_IN_PLACE: one buffer, layouts S and P alternate
    int phase = 0;         // in place: 0 = layout S (swapped), 1 = layout P (pushed)
    // LBM_BC_MLP: the network runs on a helper stream of the handle's device, concurrently with
    // the bulk step (both only read the pre-step state); events fork it from and join it to
    // the caller's stream.  Created by lbm_lee_set_closure, released by lbm_lee_destroy.
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    // LBM_BC_MLP: the history buffer holds the strips of the state before the current one;
    // false after the state was set (init, reinit, import) or the closure attached
    bool hist_valid = false;
    ~lbm_lee() {
        if (join) (void)hipEventDestroy(join);
        if (fork) (void)hipEventDestroy(fork);
        if (aux) (void)hipStreamDestroy(aux);
    }
};

namespace {

thread_local std::string g_err;

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

#define LBM_HIP(call)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) return fail(LBM_E_HIP, "%s: %s", #call, hipGetErrorString(e_));  \
    } while (0)

constexpr int kReduceBlocks = 1024;           // fixed grid of the two-pass reductions
constexpr size_t kScratchBytes = 96 * 1024;  // partials (1024 x 6 doubles) + results

size_t elem_size(int storage) {
    switch (storage) {
        case LBM_F64: return 8;
        case LBM_F32: return 4;
        case LBM_F16:
        case LBM_BF16:
        case LBM_I16:
        case LBM_E3M12: return 2;
        default: return 0;
    }
}

bool is_scaled(int storage) {
    return storage == LBM_F16 || storage == LBM_BF16 || storage == LBM_I16 || storage == LBM_E3M12;
}

bool aligned256(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

// The step kernels take their constants per shell (same |c|^2): every population of a shell
// must have the same weight f* and energy offset beta.  True for every built-in table (their
// weights are isotropic); checked here so a table that breaks it is refused, not mis-stepped.
bool shell_uniform(const LatticeTable &t) {
    double f[kShells], beta[kShells];
    bool seen[kShells] = {false, false, false, false};
    for (int i = 0; i < t.Q; ++i) {
        const int sh = t.c[i][0] * t.c[i][0] + t.c[i][1] * t.c[i][1] + t.c[i][2] * t.c[i][2];
        if (sh >= kShells) return false;
        if (!seen[sh]) {
            seen[sh] = true;
            f[sh] = t.f[i];
            beta[sh] = t.beta[i];
        } else if (f[sh] != t.f[i] || beta[sh] != t.beta[i]) {
            return false;
        }
    }
    return true;
}

int tb_tile_y(int lattice, int storage, int K);  // 0: the K-step variant has no tile shape

// One plane across the march axis (x by y in 3D, a row in 2D) in bytes of one population.
bool tb_plane_fits(const lbm_lee_desc *d, int D) {
    const double plane = (double)d->n[0] * (D == 3 ? (double)d->n[1] : 1.0) * (double)elem_size(d->storage);
    return plane < 4294967296.0;
}

lbm_status check_desc(const lbm_lee_desc *d, LatticeTable *tab) {
    if (!d) return fail(LBM_E_INVALID, "desc is NULL");
    if (!build_lattice(d->lattice, tab)) return fail(LBM_E_INVALID, "unknown lattice id %d", d->lattice);
    if (!shell_uniform(*tab)) return fail(LBM_E_UNSUPPORTED, "lattice %d: weights differ within a shell", d->lattice);
    if (elem_size(d->storage) == 0) return fail(LBM_E_INVALID, "unknown storage id %d", d->storage);
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 1 || d->n[a] > (int64_t)1 << 30) return fail(LBM_E_INVALID, "n[%d] = %lld out of range", a, (long long)d->n[a]);
        if (a >= tab->D && d->n[a] != 1) return fail(LBM_E_INVALID, "n[%d] must be 1 for a %dD lattice", a, tab->D);
    }
    const double N = (double)d->n[0] * (double)d->n[1] * (double)d->n[2];
    if (N * tab->Q > 9.0e18 / 8.0) return fail(LBM_E_INVALID, "domain too large");
    if ((double)d->n[1] * (double)d->n[2] * 16.0 > 4.0e9) return fail(LBM_E_INVALID, "too many rows (ny * nz)");
    if (!(d->tau >= 0.5) || !std::isfinite(d->tau)) return fail(LBM_E_INVALID, "tau must be finite and >= 1/2 (got %g)", d->tau);
    if (d->variant < LBM_VARIANT_AUTO || d->variant > LBM_VARIANT_OPEN2D) return fail(LBM_E_INVALID, "unknown variant %d", d->variant);
    if (d->tune < 0 || d->tune > 255) return fail(LBM_E_INVALID, "unknown tune bits 0x%x", d->tune);
    if (d->variant == LBM_VARIANT_TB2 || d->variant == LBM_VARIANT_TB3) {
        const int K = d->variant == LBM_VARIANT_TB2 ? 2 : 3;
        if (d->bc != LBM_BC_PERIODIC) return fail(LBM_E_UNSUPPORTED, "the %d-step variant needs the periodic box", K);
        if (tab->D < 2) return fail(LBM_E_UNSUPPORTED, "the %d-step variant needs a 2D or 3D lattice", K);
        if (tb_tile_y(d->lattice, d->storage, K) == 0)
            return fail(LBM_E_UNSUPPORTED, "the %d-step variant's LDS rings for lattice %d do not fit with this storage",
                        K, d->lattice);
        if (!tb_plane_fits(d, tab->D))
            return fail(LBM_E_UNSUPPORTED, "the %d-step variant addresses a plane with 32-bit byte offsets (< 4 GiB)", K);
    }
    if (d->variant == LBM_VARIANT_OPEN2D && (tab->D != 2 || d->bc == LBM_BC_PERIODIC))
        return fail(LBM_E_UNSUPPORTED, "the one-launch open-box step needs a 2D lattice and an open boundary");
    if (d->tune & kTuneInPlace) {
        if (d->bc != LBM_BC_PERIODIC) return fail(LBM_E_UNSUPPORTED, "in-place streaming needs the periodic box");
        if (d->variant != LBM_VARIANT_AUTO && d->variant != LBM_VARIANT_GENERIC)
            return fail(LBM_E_UNSUPPORTED, "in-place streaming runs its own kernels: variant must be AUTO or GENERIC");
    }
    if (!(d->store_scale >= 0.0) || !std::isfinite(d->store_scale)) return fail(LBM_E_INVALID, "store_scale must be >= 0");
    if (d->store_scale > 0.0) {
        int ex;
        if (std::frexp(d->store_scale, &ex) != 0.5) return fail(LBM_E_INVALID, "store_scale must be a power of two");
    }
    if (d->bc < LBM_BC_PERIODIC || d->bc > LBM_BC_MLP) return fail(LBM_E_INVALID, "unknown boundary %d", d->bc);
    if (d->bc != LBM_BC_PERIODIC)
        for (int a = 0; a < tab->D; ++a)
            if (d->n[a] < 3) return fail(LBM_E_INVALID, "open boundaries need n[%d] >= 3", a);
    if (d->bc == LBM_BC_SPONGE) {
        if (d->sponge_width < 1) return fail(LBM_E_INVALID, "sponge_width must be >= 1");
        if (!(d->sponge_sigma >= 0.0 && d->sponge_sigma <= 1.0)) return fail(LBM_E_INVALID, "sponge_sigma must lie in [0, 1]");
    }
    if (d->variant == LBM_VARIANT_DPP && d->n[0] % 4 != 0) return fail(LBM_E_UNSUPPORTED, "DPP variant needs nx %% 4 == 0");
    if (d->variant == LBM_VARIANT_DPP2 && d->n[0] % 2 != 0) return fail(LBM_E_UNSUPPORTED, "DPP2 variant needs nx %% 2 == 0");
    return LBM_OK;
}

// ------------------------------------------------------------------ dispatch on (velocity set, storage)
template <class VS, class F>
lbm_status visit_storage(int storage, F &&f) {
    switch (storage) {
        case LBM_F64: return f(VS{}, StF64{});
        case LBM_F32: return f(VS{}, StF32{});
        case LBM_F16: return f(VS{}, StF16{});
        case LBM_BF16: return f(VS{}, StBF16{});
        case LBM_I16: return f(VS{}, StI16{});
        case LBM_E3M12: return f(VS{}, StE3M12{});
        default: return fail(LBM_E_INVALID, "unknown storage id %d", storage);
    }
}

template <class F>
lbm_status visit(int lattice, int storage, F &&f) {
    switch (lattice) {
        case LBM_D1Q3: return visit_storage<VS_D1Q3>(storage, f);
        case LBM_D2Q5:
        case LBM_D2Q5_DIA: return visit_storage<VS_D2Q5>(storage, f);
        case LBM_D2Q9: return visit_storage<VS_D2Q9>(storage, f);
        case LBM_D3Q7:
        case LBM_D3Q7_DIA: return visit_storage<VS_D3Q7>(storage, f);
        case LBM_D3Q9: return visit_storage<VS_D3Q9>(storage, f);
        case LBM_D3Q13: return visit_storage<VS_D3Q13>(storage, f);
        case LBM_D3Q19: return visit_storage<VS_D3Q19>(storage, f);
        default: return fail(LBM_E_INVALID, "unknown lattice id %d", lattice);
    }
}

int tb_tile_y(int lattice, int storage, int K) {
    int ty = 0;
    visit(lattice, storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        if constexpr (VS::D >= 2) ty = K == 2 ? TbShape<VS, decltype(sto), 2>::TY : TbShape<VS, decltype(sto), 3>::TY;
        return LBM_OK;
    });
    return ty;
}

template <int Q>
FieldCoef<Q> field_coef(const lbm_lee *h) {
    FieldCoef<Q> k;
    const LatticeTable &t = h->tab;
    const bool scaled = is_scaled(h->desc.storage);
    for (int i = 0; i < Q; ++i) {
        k.f[i] = t.f[i];
        k.dec[i] = scaled ? t.f[i] / h->S : 1.0;
        k.enc[i] = scaled ? h->S / t.f[i] : 1.0;
        const int c2 = t.c[i][0] * t.c[i][0] + t.c[i][1] * t.c[i][1] + t.c[i][2] * t.c[i][2];
        k.e[i] = 0.5 * (c2 + t.beta[i]);
    }
    k.rho0 = t.rho0;
    k.theta0 = t.theta0;
    k.gm1 = t.gamma - 1.0;
    k.a1 = t.a1;
    k.a2 = t.a2;
    k.b = t.b;
    k.c1 = t.c1;
    k.c2 = t.c2;
    return k;
}

template <typename CT>
Kc<CT> split(double v) {
    Kc<CT> k;
    k.hi = (CT)v;
    k.lo = (CT)(v - (double)k.hi);
    return k;
}

// Per-shell collision constants (the shell of population i is |c_i|^2); shell_uniform() has
// checked that every population of a shell has the same f*_i and beta_i.
// raw_unit: the step works on stored values times raw_unit (the storage type's raw domain, 1
// for the plain formats): the moment constants take 1/raw_unit, the equilibrium weight raw_unit.
// The collision folded into two FP64 matrices per shell pair (see StepCoef): per-shell constants
// of the storage mode (scale S for the 16-bit formats, raw_unit for a raw step domain), then
// A = kA rho' + kA' e and C = kC rho' + kC' e after eliminating theta'.
void fold_constants(const LatticeTable &t, int storage, double S, double tau, double raw_unit,
                    double H[kShells][kShells], double WB[kShells][kShells], double &keep) {
    const bool scaled = is_scaled(storage);
    const double omega = 1.0 / tau;
    double dec[kShells] = {}, edec[kShells] = {}, bu[kShells] = {}, w[kShells] = {};
    for (int i = 0; i < t.Q; ++i) {  // shell_uniform() has checked that a shell's constants agree
        const int sh = t.c[i][0] * t.c[i][0] + t.c[i][1] * t.c[i][1] + t.c[i][2] * t.c[i][2];
        const double d = scaled ? t.f[i] / S : 1.0, e = scaled ? S / t.f[i] : 1.0;
        dec[sh] = d / raw_unit;
        edec[sh] = 0.5 * (sh + t.beta[i]) * d / raw_unit;
        bu[sh] = t.b * d / t.rho0 / raw_unit;
        w[sh] = omega * e * t.f[i] * raw_unit;
    }
    const double gm1_rho0 = (t.gamma - 1.0) / t.rho0, theta0_rho0 = t.theta0 / t.rho0;
    const double kA = t.a1 - t.a2 * theta0_rho0, kAe = t.a2 * gm1_rho0;
    const double kC = t.c1 - t.c2 * theta0_rho0, kCe = t.c2 * gm1_rho0;
    for (int to = 0; to < kShells; ++to)
        for (int from = 0; from < kShells; ++from) {
            const double gA = kA * dec[from] + kAe * edec[from], gC = kC * dec[from] + kCe * edec[from];
            H[to][from] = w[to] * (gA + 0.5 * to * gC);
            WB[to][from] = w[to] * bu[from];
        }
    keep = 1.0 - omega;
}

template <typename CT, int Q>
StepCoef<CT, Q> step_coef(const lbm_lee *h, double raw_unit = 1.0) {
    StepCoef<CT, Q> k;
    std::memset(&k, 0, sizeof k);
    double H[kShells][kShells], WB[kShells][kShells], keep;
    fold_constants(h->tab, h->desc.storage, h->S, h->desc.tau, raw_unit, H, WB, keep);
    for (int to = 0; to < kShells; ++to)
        for (int from = 0; from < kShells; ++from) {
            k.H[to][from] = split<CT>(H[to][from]);
            k.WB[to][from] = split<CT>(WB[to][from]);
        }
    k.keep = split<CT>(keep);
    return k;
}

// Face frames: negate axis a for the high side, then swap axis a with x, so the outward normal
// becomes -x.  perm[f][j]: population whose transformed velocity is canonical velocity j.
template <class VS>
FaceTab<VS::Q> face_table(const LatticeTable &t, const int64_t n[3]) {
    FaceTab<VS::Q> ft;
    std::memset(&ft, 0, sizeof ft);
    ft.D = t.D;
    ft.nfaces = 2 * t.D;
    for (int a = 0; a < 3; ++a) ft.n[a] = (int)n[a];
    long long off = 0;
    for (int f = 0; f < ft.nfaces; ++f) {
        const int a = f >> 1, side = f & 1;
        ft.node_off[f] = off;
        long long cnt = 1;
        for (int b = 0; b < t.D; ++b)
            if (b != a) cnt *= n[b];
        off += cnt;
        for (int i = 0; i < VS::Q; ++i) ft.rank[f][i] = -1;
        for (int i = 0; i < VS::Q; ++i) {
            int c[3] = {t.c[i][0], t.c[i][1], t.c[i][2]};
            if (side) c[a] = -c[a];
            const int tmp = c[0];
            c[0] = c[a];
            c[a] = tmp;
            for (int j = 0; j < VS::Q; ++j)
                if (t.c[j][0] == c[0] && t.c[j][1] == c[1] && t.c[j][2] == c[2]) ft.perm[f][j] = (signed char)i;
        }
        for (int r = 0; r < NetGeom<VS>::NOUT; ++r) ft.rank[f][ft.perm[f][entering_index<VS>(r)]] = (signed char)r;
    }
    for (int f = ft.nfaces; f < 7; ++f) ft.node_off[f] = off;
    return ft;
}

// The rest population (index 0, velocity 0) is invariant under the update for every tau when
// the equilibrium map E = d g^eq / d g has E_00 = 1 and E_0j = E_j0 = 0: then
// g_0* = (1 - 1/tau) g_0 + (1/tau) g_0 = g_0 and no moving population depends on g_0.  The
// sponge damps every population, so it keeps the rest population in the update.
bool rest_decoupled(const LatticeTable &t) {
    if (t.c[0][0] || t.c[0][1] || t.c[0][2]) return false;
    auto E = [&](int i, int j) {
        const int c2i = t.c[i][0] * t.c[i][0] + t.c[i][1] * t.c[i][1] + t.c[i][2] * t.c[i][2];
        const int c2j = t.c[j][0] * t.c[j][0] + t.c[j][1] * t.c[j][1] + t.c[j][2] * t.c[j][2];
        const int cc = t.c[i][0] * t.c[j][0] + t.c[i][1] * t.c[j][1] + t.c[i][2] * t.c[j][2];
        const double wth = ((t.gamma - 1.0) * 0.5 * (c2j + t.beta[j]) - t.theta0) / t.rho0;
        return t.f[i] * ((t.a1 + 0.5 * c2i * t.c1) + t.b * cc / t.rho0 + wth * (t.a2 + 0.5 * c2i * t.c2));
    };
    if (std::fabs(E(0, 0) - 1.0) > 1e-12) return false;
    for (int j = 1; j < t.Q; ++j)
        if (std::fabs(E(0, j)) > 1e-12 || std::fabs(E(j, 0)) > 1e-12) return false;
    return true;
}

bool skip_rest(const LatticeTable &t, const lbm_lee_desc *d) {
    return rest_decoupled(t) && d->bc != LBM_BC_SPONGE && !(d->tune & LBM_TUNE_FULL_REST);
}

int64_t face_node_count(const LatticeTable &t, const int64_t n[3]) {
    int64_t total = 0;
    for (int a = 0; a < t.D; ++a) {
        int64_t cnt = 1;
        for (int b = 0; b < t.D; ++b)
            if (b != a) cnt *= n[b];
        total += 2 * cnt;
    }
    return total;
}

int net_outputs(const LatticeTable &t) {
    int k = 0;
    for (int i = 0; i < t.Q; ++i) k += t.c[i][0] == 1 ? 1 : 0;
    return k;
}

int64_t net_inputs(const LatticeTable &t) { return (int64_t)kHistory * 3 * t.Q; }

int64_t net_params(const LatticeTable &t) {
    const int64_t nin = net_inputs(t), nout = net_outputs(t);
    return nin * kHidden + kHidden + kHidden * kHidden + kHidden + kHidden * nout + nout;
}

unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

lbm_status launch_check() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LBM_E_HIP, "kernel launch: %s", hipGetErrorString(e));
    return LBM_OK;
}

// AUTO: measured on MI355X (D3Q7, 256^3): the temporal-blocking variants beat every one-step
// kernel on large periodic boxes (they move the state through HBM once per two or three
// steps), three steps beating two except for D3Q19; below a million cells the launches are
// short and the one-step kernels win.  Of the one-step kernels
// the one-cell-per-thread gather has the highest occupancy and wins for 4- and 8-byte storage;
// 2-byte storage needs wider per-lane accesses.
int resolve_variant(const lbm_lee *h) {
    if (h->inplace) return LBM_VARIANT_GENERIC;  // the in-place kernels are one thread per cell
    if (h->desc.variant != LBM_VARIANT_AUTO) return h->desc.variant;
    // 2D open boxes: ring, interior and closure network in one launch (the separate kernels of
    // the other variants are each latency-bound on boxes of this size)
    if (h->desc.bc != LBM_BC_PERIODIC && h->tab.D == 2) return LBM_VARIANT_OPEN2D;
    // periodic boxes of a million cells and more: three steps per launch for the sets of up to 9
    // velocities, two for the larger ones (their two collisions per column already fill the
    // registers), for every storage mode
    if (h->desc.bc == LBM_BC_PERIODIC && h->tab.D >= 2 && h->N >= ((size_t)1 << 20) && tb_plane_fits(&h->desc, h->tab.D)) {
        if (h->tab.Q <= 9 && tb_tile_y(h->desc.lattice, h->desc.storage, 3) > 0) return LBM_VARIANT_TB3;
        if (tb_tile_y(h->desc.lattice, h->desc.storage, 2) > 0) return LBM_VARIANT_TB2;
    }
    if (elem_size(h->desc.storage) >= 4) return LBM_VARIANT_GENERIC;
    if (h->nx % 4 == 0) return LBM_VARIANT_DPP;
    if (h->nx % 2 == 0) return LBM_VARIANT_DPP2;
    return LBM_VARIANT_GENERIC;
}

// Layout of the state buffer as it is now, and the one a fresh state is written in.
Layout layout_now(const lbm_lee *h) {
    Layout l{kLayoutPlain, h->nx, h->ny, h->nz};
    if (h->inplace) l.mode = h->phase == 0 ? kLayoutSwapped : kLayoutPushed;
    return l;
}
Layout layout_fresh(const lbm_lee *h) {
    Layout l{h->inplace ? kLayoutSwapped : kLayoutPlain, h->nx, h->ny, h->nz};
    return l;
}
// The other ping-pong buffer's rest plane (kept equal to this one's when the step skips it).
void *rest_copy_buffer(const lbm_lee *h) { return (h->skip0 && !h->inplace) ? h->buf[h->cur ^ 1] : nullptr; }

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
    const int variant = resolve_variant(h);
    const int bc = h->desc.bc;
    if (bc == LBM_BC_MLP && (!h->net || !h->ghost))
        return fail(LBM_E_STATE, "an LBM_BC_MLP handle needs lbm_lee_set_closure before stepping");
    lbm_status s = visit(h->desc.lattice, h->desc.storage, [&](auto vs, auto sto) -> lbm_status {
        using VS = decltype(vs);
        using ST = decltype(sto);
        using E = typename ST::elem;
        // bulk kernels in the storage type's raw domain; the shell recompute in the real one
        const auto k = step_coef<typename ST::comp, VS::Q>(h, ST::raw_unit);
        const auto ks = step_coef<typename ST::comp, VS::Q>(h);
        const int vec = variant == LBM_VARIANT_DPP2 ? 2 : 4;
        const int cpr = (h->nx + 64 * vec - 1) / (64 * vec);
        const unsigned waves = (unsigned)((size_t)h->ny * h->nz * cpr);
        const bool fullrow = h->nx == 64 * vec;
        const unsigned tune = (unsigned)h->desc.tune;
        const bool fork = (tune & 16u) != 0;  // LBM_TUNE_CLOSURE_STREAM
        const unsigned full_grid = (waves + 3) / 4;
        // persistent DPP launches: the grid is the resident block slots of the exact kernel launched
        auto dpp_grid = [&](const void *fn) -> unsigned {
            if (!(tune & kTunePersistent) || h->cus <= 0) return full_grid;
            int per_cu = 0;
            unsigned g = full_grid;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) == hipSuccess && per_cu > 0)
                g = std::min(g, (unsigned)(per_cu * h->cus));
            (void)hipGetLastError();
            return g;
        };
        const int lds_cpr = (h->nx + 255) / 256;
        const unsigned lds_blocks = (unsigned)((size_t)h->ny * h->nz * lds_cpr);
        FaceTab<VS::Q> ft;
        FieldCoef<VS::Q> fk;
        unsigned shell_x = 1, ghost_blocks = 1, sponge_x = 1;
        long long nodes = 0;
        const long long nstrip = 3 * VS::Q;
        if (bc != LBM_BC_PERIODIC) {
            ft = face_table<VS>(h->tab, h->desc.n);
            fk = field_coef<VS::Q>(h);
            long long mx = 1;
            for (int a = 0; a < VS::D; ++a) {
                long long cnt = 1;
                for (int b = 0; b < VS::D; ++b)
                    if (b != a) cnt *= h->desc.n[b];
                if (cnt > mx) mx = cnt;
            }
            shell_x = (unsigned)((mx + 255) / 256);
            if (bc == LBM_BC_SPONGE) {  // the largest slab: depth W times a full face
                long long big = 1;
                for (int a = 0; a < VS::D; ++a) {
                    long long cnt = std::min<long long>(h->desc.sponge_width, h->desc.n[a]);
                    for (int b = 0; b < VS::D; ++b)
                        if (b != a) cnt *= h->desc.n[b];
                    big = std::max(big, cnt);
                }
                sponge_x = (unsigned)((big + 255) / 256);
            }
            nodes = ft.node_off[ft.nfaces];
            const long long tiles = (nodes + 15) / 16;
            ghost_blocks = (unsigned)std::min<long long>((tiles + 3) / 4, 4096);
        }
        auto run = [&](auto skip, auto half) -> lbm_status {
            constexpr bool SK = decltype(skip)::value;
            constexpr bool HF = decltype(half)::value;
            const bool dpp = variant == LBM_VARIANT_DPP || variant == LBM_VARIANT_DPP2;
            const unsigned g_dpp4t = dpp && vec == 4 && fullrow ? dpp_grid((const void *)&step_dpp<VS, ST, 4, true, SK, HF>) : 1;
            const unsigned g_dpp4f = dpp && vec == 4 && !fullrow ? dpp_grid((const void *)&step_dpp<VS, ST, 4, false, SK, HF>) : 1;
            const unsigned g_dpp2t = dpp && vec == 2 && fullrow ? dpp_grid((const void *)&step_dpp<VS, ST, 2, true, SK, HF>) : 1;
            const unsigned g_dpp2f = dpp && vec == 2 && !fullrow ? dpp_grid((const void *)&step_dpp<VS, ST, 2, false, SK, HF>) : 1;
            if (h->inplace) {  // periodic box, one buffer: layouts S and P alternate
                E *A = static_cast<E *>(h->buf[0]);
                for (int64_t t = 0; t < nsteps; ++t) {
                    if (h->phase == 0)
                        step_inplace<VS, ST, SK, HF, true><<<blocks_for(h->N), 256, 0, st>>>(A, h->nx, h->ny, h->nz,
                                                                                          h->N, k);
                    else
                        step_inplace<VS, ST, SK, HF, false><<<blocks_for(h->N), 256, 0, st>>>(A, h->nx, h->ny, h->nz,
                                                                                           h->N, k);
                    lbm_status ls = launch_check();
                    if (ls != LBM_OK) return ls;
                    h->phase ^= 1;
                    h->steps += 1;
                }
                return LBM_OK;
            }
            // periodic box, K steps per launch; a remainder of the step count runs one-step launches
            auto run_tbk = [&](auto kk) -> lbm_status {
                constexpr int K = decltype(kk)::value;
                if constexpr (VS::D >= 2) {
                    using SH = TbShape<VS, ST, K>;
                    if constexpr (SH::TY > 0) {
                        const int fx = h->nx, fy = VS::D == 3 ? h->ny : 1, fz = VS::D == 3 ? h->nz : h->ny;
                        const long long tiles_x = (fx + kTbTx - 1) / kTbTx, tiles_y = (fy + SH::TY - 1) / SH::TY;
                        auto fn = step_tbk<VS, ST, SK, HF, K, SH::TY, SH::NT, SH::WPE>;
                        int sz = 16;
                        const unsigned seg_bits = (tune >> 6) & 3u;
                        if (seg_bits) {
                            sz = 4 << seg_bits;  // 8, 16, 32
                        } else {
                            // a block's time is about proportional to the planes it computes
                            // (sz + 2(K - 1)); the grid runs in ceil(blocks / resident slots) rounds
                            int per_cu = 0;
                            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)fn, SH::NT, 0) !=
                                    hipSuccess || per_cu <= 0)
                                per_cu = 1;
                            (void)hipGetLastError();
                            const long long slots = (long long)std::max(h->cus, 1) * per_cu;
                            long long best = -1;
                            for (int cand = 4; cand <= 64; ++cand) {
                                const long long g = tiles_x * tiles_y * ((fz + cand - 1) / cand);
                                const long long cost = ((g + slots - 1) / slots) * (std::min(cand, fz) + 2 * (K - 1));
                                if (best < 0 || cost < best) {
                                    best = cost;
                                    sz = cand;
                                }
                            }
                        }
                        const long long blocks = tiles_x * tiles_y * ((fz + sz - 1) / sz);
                        int64_t t = 0;
                        for (; t + K <= nsteps; t += K) {
                            const E *src = static_cast<const E *>(h->buf[h->cur]);
                            E *dst = static_cast<E *>(h->buf[h->cur ^ 1]);
                            fn<<<(unsigned)blocks, SH::NT, 0, st>>>(src, dst, fx, fy, fz, h->N, sz, (int)tiles_x,
                                                                   (int)tiles_y, k);
                            lbm_status ls = launch_check();
                            if (ls != LBM_OK) return ls;
                            h->cur ^= 1;
                            h->steps += K;
                        }
                        for (; t < nsteps; ++t) {
                            const E *src = static_cast<const E *>(h->buf[h->cur]);
                            E *dst = static_cast<E *>(h->buf[h->cur ^ 1]);
                            step_generic<VS, ST, SK, HF><<<blocks_for(h->N), 256, 0, st>>>(src, dst, h->nx, h->ny, h->nz,
                                                                                        h->N, k);
                            lbm_status ls = launch_check();
                            if (ls != LBM_OK) return ls;
                            h->cur ^= 1;
                            h->steps += 1;
                        }
                        return LBM_OK;
                    }
                }
                return fail(LBM_E_UNSUPPORTED, "the %d-step variant does not support this lattice and storage", K);
            };
            if (variant == LBM_VARIANT_OPEN2D) {
                if constexpr (VS::D == 2) {
                    const int nx = h->nx, ny = h->ny;
                    const long long ring = 2LL * ny + 2LL * (nx - 2);
                    const unsigned face_blocks = bc == LBM_BC_MLP ? (unsigned)((open2d_segments(nx, ny) + 3) / 4)
                                                                  : (unsigned)((ring + 255) / 256);
                    const long long interior = (long long)(nx - 2) * (ny - 2);
                    const unsigned bulk_blocks =
                        (unsigned)std::min<long long>((interior + 256 * kOpenCells - 1) / (256 * kOpenCells), 1LL << 20);
                    for (int64_t t = 0; t < nsteps; ++t) {
                        const E *src = static_cast<const E *>(h->buf[h->cur]);
                        E *dst = static_cast<E *>(h->buf[h->cur ^ 1]);
                        if (bc == LBM_BC_MLP) {
                            float *hist = h->ghost + nodes * (long long)net_outputs(h->tab);
                            const float *hin = h->hist_valid ? hist + (long long)h->cur * nodes * nstrip : nullptr;
                            float *hout = hist + (long long)(h->cur ^ 1) * nodes * nstrip;
                            open_step_2d<VS, ST, SK, HF, true><<<face_blocks + bulk_blocks, 256, 0, st>>>(
                                src, dst, h->N, bc, (int)face_blocks, h->net, h->ghost, hin, hout, ft, k, ks, fk, 0,
                                0.0);
                            h->hist_valid = true;
                        } else {
                            // the sponge layer is damped inside the step kernel
                            open_step_2d<VS, ST, SK, HF, false><<<face_blocks + bulk_blocks, 256, 0, st>>>(
                                src, dst, h->N, bc, (int)face_blocks, nullptr, nullptr, nullptr, nullptr, ft, k, ks, fk,
                                bc == LBM_BC_SPONGE ? h->desc.sponge_width : 0, h->desc.sponge_sigma);
                        }
                        lbm_status ls = launch_check();
                        if (ls != LBM_OK) return ls;
                        h->cur ^= 1;
                        h->steps += 1;
                    }
                    return LBM_OK;
                }
                return fail(LBM_E_UNSUPPORTED, "the one-launch open-box step needs a 2D lattice");
            }
            if (variant == LBM_VARIANT_TB2) return run_tbk(std::integral_constant<int, 2>{});
            if (variant == LBM_VARIANT_TB3) return run_tbk(std::integral_constant<int, 3>{});
            for (int64_t t = 0; t < nsteps; ++t) {
                const E *src = static_cast<const E *>(h->buf[h->cur]);
                E *dst = static_cast<E *>(h->buf[h->cur ^ 1]);
                if (bc == LBM_BC_MLP) {
                    // history pair after the ghost values, selected by the state buffer's parity
                    float *hist = h->ghost + nodes * (long long)net_outputs(h->tab);
                    const float *hin = h->hist_valid ? hist + (long long)h->cur * nodes * nstrip : nullptr;
                    float *hout = hist + (long long)(h->cur ^ 1) * nodes * nstrip;
                    if (fork) {  // fork: the network on the helper stream
                        LBM_HIP(hipEventRecord(h->fork, st));
                        LBM_HIP(hipStreamWaitEvent(h->aux, h->fork, 0));
                    }
                    if (hin)
                        ghost_mlp_kernel<VS, ST, true><<<ghost_blocks, 256, 0, fork ? h->aux : st>>>(
                            src, h->N, h->net, h->ghost, hin, hout, ft, fk);
                    else
                        ghost_mlp_kernel<VS, ST, false><<<ghost_blocks, 256, 0, fork ? h->aux : st>>>(
                            src, h->N, h->net, h->ghost, hin, hout, ft, fk);
                    if (fork) LBM_HIP(hipEventRecord(h->join, h->aux));
                    h->hist_valid = true;
                }
                if (variant == LBM_VARIANT_GENERIC) {
                    step_generic<VS, ST, SK, HF><<<blocks_for(h->N), 256, 0, st>>>(src, dst, h->nx, h->ny, h->nz, h->N, k);
                } else if (variant == LBM_VARIANT_LDS) {
                    step_lds<VS, ST, SK, HF><<<lds_blocks, 256, 0, st>>>(src, dst, h->nx, h->ny, h->nz, h->N, lds_cpr, k);
                } else if (vec == 4) {
                    if (fullrow)
                        step_dpp<VS, ST, 4, true, SK, HF><<<g_dpp4t, 256, 0, st>>>(src, dst, h->nx, h->ny, h->nz, h->N,
                                                                              cpr, waves, tune, k);
                    else
                        step_dpp<VS, ST, 4, false, SK, HF><<<g_dpp4f, 256, 0, st>>>(src, dst, h->nx, h->ny, h->nz, h->N,
                                                                               cpr, waves, tune, k);
                } else {
                    if (fullrow)
                        step_dpp<VS, ST, 2, true, SK, HF><<<g_dpp2t, 256, 0, st>>>(src, dst, h->nx, h->ny, h->nz, h->N,
                                                                              cpr, waves, tune, k);
                    else
                        step_dpp<VS, ST, 2, false, SK, HF><<<g_dpp2f, 256, 0, st>>>(src, dst, h->nx, h->ny, h->nz, h->N,
                                                                               cpr, waves, tune, k);
                }
                if (bc == LBM_BC_MLP && fork) LBM_HIP(hipStreamWaitEvent(st, h->join, 0));  // join
                if (bc != LBM_BC_PERIODIC) {
                    shell_kernel<VS, ST, SK, HF><<<dim3(shell_x, 2 * VS::D), 256, 0, st>>>(src, dst, h->N, bc, h->ghost,
                                                                                      ft, ks, fk);
                    if (bc == LBM_BC_SPONGE)
                        sponge_kernel<VS, ST><<<dim3(sponge_x, 2 * VS::D), 256, 0, st>>>(
                            dst, h->N, h->nx, h->ny, h->nz, h->desc.sponge_width, h->desc.sponge_sigma);
                }
                lbm_status ls = launch_check();
                if (ls != LBM_OK) return ls;
                h->cur ^= 1;
                h->steps += 1;
            }
            return LBM_OK;
        };
        // tau = 1/2 (keep = 1 - 1/tau = -1) takes the shorter relaxation s <- w t - s, which
        // gives the same bits as the general form with keep = -1 in fewer operations.
        if (h->desc.tau == 0.5) {
            if constexpr (VS::rest_may_decouple) {
                if (h->skip0) return run(std::true_type{}, std::true_type{});
            }
            return run(std::false_type{}, std::true_type{});
        }
        if constexpr (VS::rest_may_decouple) {
            if (h->skip0) return run(std::true_type{}, std::false_type{});
        }
        return run(std::false_type{}, std::false_type{});
    });
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
        nrbc_forward_kernel<VS><<<grid, 256, 0, st>>>(params, strips, count, out);
        return launch_check();
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

lbm_status lbm_lee_compare_fields(const double *a, const int64_t n_a[3], const double *b, const int64_t n_b[3],
                                  const int64_t origin[3], double out[3], void *scratch, size_t scratch_bytes,
                                  void *stream) {
    if (!a || !n_a || !b || !n_b || !origin || !out || !scratch) return fail(LBM_E_INVALID, "bad arguments");
    if (scratch_bytes < kScratchBytes || !aligned256(scratch)) return fail(LBM_E_INVALID, "scratch too small or misaligned");
    for (int d = 0; d < 3; ++d)
        if (n_a[d] < 1 || origin[d] < 0 || origin[d] + n_a[d] > n_b[d] || n_a[d] > (1 << 30) || n_b[d] > (1 << 30))
            return fail(LBM_E_INVALID, "box a must lie inside box b (axis %d)", d);
    hipStream_t st = static_cast<hipStream_t>(stream);
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
    return ok();
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
