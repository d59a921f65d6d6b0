// Internal declarations shared by the library's translation units: the handle, argument
// checks, the dispatch over (velocity set, storage), the host-side constant folding.  Not part of
// the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>

#include "../../include/lbm_lee.h"
#include "kernels.hpp"
#include "nrbc.hpp"
#include "open_bc.hpp"
#include "tables.hpp"
#include "resident.hpp"
#include "temporal.hpp"

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

namespace lbm {
namespace api {

// Record an error message for lbm_lee_last_error() and return st (defined in api.hip).
lbm_status fail(lbm_status st, const char *fmt, ...);
lbm_status ok();

#define LBM_HIP(call)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) return fail(LBM_E_HIP, "%s: %s", #call, hipGetErrorString(e_));  \
    } while (0)

constexpr int kReduceBlocks = 1024;           // fixed grid of the two-pass reductions
constexpr size_t kScratchBytes = 96 * 1024;  // partials (1024 x 6 doubles) + results

inline size_t elem_size(int storage) {
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

inline bool is_scaled(int storage) {
    return storage == LBM_F16 || storage == LBM_BF16 || storage == LBM_I16 || storage == LBM_E3M12;
}

inline bool aligned256(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

// The step kernels take their constants per shell (same |c|^2): every population of a shell
// must have the same weight f* and energy offset beta.  True for every built-in table (their
// weights are isotropic); checked here so a table that breaks it is refused, not mis-stepped.
inline bool shell_uniform(const LatticeTable &t) {
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

inline int tb_tile_y(int lattice, int storage, int K);  // 0: the K-step variant has no tile shape

// One plane across the march axis (x by y in 3D, a row in 2D) in bytes of one population: the
// multi-step kernels address it with 32-bit offsets and keep 2^31 and above for "out of range".
inline bool tb_plane_fits(const lbm_lee_desc *d, int D) {
    const double plane = (double)d->n[0] * (D == 3 ? (double)d->n[1] : 1.0) * (double)elem_size(d->storage);
    return plane <= 2147483648.0;
}

// The closure network's matrix-core tiles: at most 128 inputs (6 Q) and 16 outputs.
inline bool net_fits(const LatticeTable &t) {
    int k = 0;
    for (int i = 0; i < t.Q; ++i) k += t.c[i][0] == 1 ? 1 : 0;
    return (kHistory * 3 * t.Q + 31) / 32 * 32 <= 128 && k <= 16;  // as NetGeom::fits
}

// A damped layer along the faces: the sponge closure's, and the network closure's when it is
// given a width (a network behind a sponge layer).
inline bool sponge_layer(const lbm_lee_desc *d) {
    return d->bc == LBM_BC_SPONGE || (d->bc == LBM_BC_MLP && d->sponge_width > 0);
}

// Two copies of the whole state fit the LDS-resident step's 160 KiB.
inline bool resident_fits(const lbm_lee_desc *d, const LatticeTable &t) {
    const double cells = (double)d->n[0] * (double)d->n[1] * (double)d->n[2];
    return 2.0 * t.Q * cells * (double)elem_size(d->storage) <= (double)kResidentLds;
}

inline lbm_status check_desc(const lbm_lee_desc *d, LatticeTable *tab) {
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
    if (d->variant < LBM_VARIANT_AUTO || d->variant > LBM_VARIANT_RESIDENT) return fail(LBM_E_INVALID, "unknown variant %d", d->variant);
    if (d->variant == LBM_VARIANT_RESIDENT) {
        if (d->bc != LBM_BC_PERIODIC) return fail(LBM_E_UNSUPPORTED, "the LDS-resident variant needs the periodic box");
        if (!resident_fits(d, *tab))
            return fail(LBM_E_UNSUPPORTED, "the LDS-resident variant holds two copies of the state in 160 KiB");
    }
    if (d->tune < 0 || d->tune > 511) return fail(LBM_E_INVALID, "unknown tune bits 0x%x", d->tune);
    if (d->variant == LBM_VARIANT_TB2 || d->variant == LBM_VARIANT_TB3) {
        const int K = d->variant == LBM_VARIANT_TB2 ? 2 : 3;
        if (d->bc != LBM_BC_PERIODIC) return fail(LBM_E_UNSUPPORTED, "the %d-step variant needs the periodic box", K);
        if (tab->D < 2) return fail(LBM_E_UNSUPPORTED, "the %d-step variant needs a 2D or 3D lattice", K);
        if (tb_tile_y(d->lattice, d->storage, K) == 0)
            return fail(LBM_E_UNSUPPORTED, "the %d-step variant's LDS rings for lattice %d do not fit with this storage",
                        K, d->lattice);
        if (tab->D == 3 && d->n[0] % 2 != 0)
            return fail(LBM_E_UNSUPPORTED, "the %d-step variant reads and writes x-pairs in 3D: nx must be even", K);
        if (!tb_plane_fits(d, tab->D))
            return fail(LBM_E_UNSUPPORTED, "the %d-step variant addresses a plane with 31-bit byte offsets (<= 2 GiB)", K);
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
    if (d->bc == LBM_BC_MLP && !net_fits(*tab))
        return fail(LBM_E_UNSUPPORTED, "the closure network takes sets of up to 21 velocities (lattice %d has %d)",
                    d->lattice, tab->Q);
    if (d->bc == LBM_BC_SPONGE && d->sponge_width < 1) return fail(LBM_E_INVALID, "sponge_width must be >= 1");
    if (d->bc == LBM_BC_MLP && d->sponge_width < 0)
        return fail(LBM_E_INVALID, "sponge_width must be >= 0 with the network closure");
    if (sponge_layer(d) && !(d->sponge_sigma >= 0.0 && d->sponge_sigma <= 1.0))
        return fail(LBM_E_INVALID, "sponge_sigma must lie in [0, 1]");
    if (d->variant == LBM_VARIANT_DPP && d->n[0] % 4 != 0) return fail(LBM_E_UNSUPPORTED, "DPP variant needs nx %% 4 == 0");
    if (d->variant == LBM_VARIANT_DPP2 && d->n[0] % 2 != 0) return fail(LBM_E_UNSUPPORTED, "DPP2 variant needs nx %% 2 == 0");
    return LBM_OK;
}

// ------------------------------------------------------------------ dispatch on (velocity set, storage)
template <class VS, class F>
inline lbm_status visit_storage(int storage, F &&f) {
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
inline lbm_status visit(int lattice, int storage, F &&f) {
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
        case LBM_D3Q27: return visit_storage<VS_D3Q27>(storage, f);
        default: return fail(LBM_E_INVALID, "unknown lattice id %d", lattice);
    }
}

inline int tb_tile_y(int lattice, int storage, int K) {
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
inline void fold_constants(const LatticeTable &t, int storage, double S, double tau, double raw_unit,
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
        for (int r = 0; r < entering_count<VS>(); ++r) ft.rank[f][ft.perm[f][entering_index<VS>(r)]] = (signed char)r;
    }
    for (int f = ft.nfaces; f < 7; ++f) ft.node_off[f] = off;
    return ft;
}

// The rest population (index 0, velocity 0) is invariant under the update for every tau when
// the equilibrium map E = d g^eq / d g has E_00 = 1 and E_0j = E_j0 = 0: then
// g_0* = (1 - 1/tau) g_0 + (1/tau) g_0 = g_0 and no moving population depends on g_0.  A
// sponge layer damps every population, so it keeps the rest population in the update.
inline bool rest_decoupled(const LatticeTable &t) {
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

inline bool skip_rest(const LatticeTable &t, const lbm_lee_desc *d) {
    return rest_decoupled(t) && !sponge_layer(d) && !(d->tune & LBM_TUNE_FULL_REST);
}

inline int64_t face_node_count(const LatticeTable &t, const int64_t n[3]) {
    int64_t total = 0;
    for (int a = 0; a < t.D; ++a) {
        int64_t cnt = 1;
        for (int b = 0; b < t.D; ++b)
            if (b != a) cnt *= n[b];
        total += 2 * cnt;
    }
    return total;
}

inline int net_outputs(const LatticeTable &t) {
    int k = 0;
    for (int i = 0; i < t.Q; ++i) k += t.c[i][0] == 1 ? 1 : 0;
    return k;
}

inline int64_t net_inputs(const LatticeTable &t) { return (int64_t)kHistory * 3 * t.Q; }

inline int64_t net_params(const LatticeTable &t) {
    const int64_t nin = net_inputs(t), nout = net_outputs(t);
    return nin * kHidden + kHidden + kHidden * kHidden + kHidden + kHidden * nout + nout;
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

inline lbm_status launch_check() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LBM_E_HIP, "kernel launch: %s", hipGetErrorString(e));
    return LBM_OK;
}

// AUTO: measured on MI355X.  The temporal-blocking variants beat every one-step kernel on large
// periodic boxes (they move the state through HBM once per two or three steps), three steps
// beating two except for D3Q19, and on mid-size ones (fewer launches); on small boxes the
// one-cell-per-thread step, which has the highest occupancy, wins in every storage.  Open boxes
// have their own kernels (one launch per step in 2D, the bulk step closing the x faces in 3D).
inline int resolve_variant(const lbm_lee *h) {
    if (h->inplace) return LBM_VARIANT_GENERIC;  // the in-place kernels are one thread per cell
    if (h->desc.variant != LBM_VARIANT_AUTO) return h->desc.variant;
    // tiny periodic boxes: every step of a call in one launch, the state in LDS
    if (h->desc.bc == LBM_BC_PERIODIC && resident_fits(&h->desc, h->tab)) return LBM_VARIANT_RESIDENT;
    // 2D open boxes: ring, interior and closure network in one launch up to 8 M cells (the
    // separate kernels of the other variants are each latency-bound there); on larger boxes the
    // one-launch kernel's interior blocks, which reserve the network's LDS, lose to the
    // one-cell-per-thread step plus the boundary kernels (D2Q9, us per step, one launch against
    // separate kernels: 2048^2 FP32 network 62 vs 81, E3M12 31 vs 51; 4096^2 FP32 zero 259 vs
    // 222, network 252 vs 237, E3M12 about equal)
    if (h->desc.bc != LBM_BC_PERIODIC && h->tab.D == 2)
        return h->N <= ((size_t)8 << 20) ? LBM_VARIANT_OPEN2D : LBM_VARIANT_GENERIC;
    // periodic boxes of a million cells and more: three steps per launch for the sets of up to 9
    // velocities, two for the larger ones (their two collisions per column already fill the
    // registers), for every storage mode
    if (h->desc.bc == LBM_BC_PERIODIC && h->tab.D >= 2 && h->N >= ((size_t)1 << 20) && tb_plane_fits(&h->desc, h->tab.D) &&
        (h->tab.D == 2 || h->nx % 2 == 0)) {
        if (h->tab.Q <= 9 && tb_tile_y(h->desc.lattice, h->desc.storage, 3) > 0) return LBM_VARIANT_TB3;
        // (not for 2-byte storage: D3Q13 256^3, us per step, TB2 / DPP, FP16 172 / 147, BF16 173 / 140)
        if (elem_size(h->desc.storage) != 2 && tb_tile_y(h->desc.lattice, h->desc.storage, 2) > 0)
            return LBM_VARIANT_TB2;
    }
    // periodic 2D boxes of 2^18 to 2^20 cells: two steps per launch (the launches, not HBM, bound a
    // step there; D2Q9 512^2, us per step, GENERIC / DPP / TB2 / TB3: FP32 7.7 / 6.0 / 4.2 / 4.8,
    // FP16 4.9 / 4.6 / 4.0 / 4.2; D2Q5 FP32 4.3 / 3.4 / 2.9 / 2.7; at 256^2 all within 1 us)
    if (h->desc.bc == LBM_BC_PERIODIC && h->tab.D == 2 && h->N >= ((size_t)1 << 18) && tb_plane_fits(&h->desc, 2) &&
        tb_tile_y(h->desc.lattice, h->desc.storage, 2) > 0)
        return LBM_VARIANT_TB2;
    // periodic 3D boxes of 3 x 2^18 cells and more, sets of up to 9 velocities: three steps per launch
    // (D3Q7 96^3, us per step, GENERIC / TB3: FP32 8.4 / 7.6, FP16 8.3 / 6.0, FP64 14.0 / 8.6; at
    // 64^3 GENERIC is ahead)
    if (h->desc.bc == LBM_BC_PERIODIC && h->tab.D == 3 && h->N >= ((size_t)3 << 18) && h->tab.Q <= 9 &&
        h->nx % 2 == 0 && tb_plane_fits(&h->desc, 3) && tb_tile_y(h->desc.lattice, h->desc.storage, 3) > 0)
        return LBM_VARIANT_TB3;
    // 3D open boxes: the DPP bulk step closes the x faces (and damps a sponge layer) itself, which
    // beats the one-cell-per-thread step plus the full boundary pass for every set and storage but
    // D3Q27 with 8-byte storage, whose DPP kernel spills (ms per step, GENERIC against DPP; D3Q7
    // 384^3: FP32 zero 0.611 / 0.508, network 0.749 / 0.671, sponge W 16 0.907 / 0.599; FP64 zero
    // 1.120 / 1.023; 256^3 zero closure, FP32 / FP64: D3Q9 0.258 / 0.212, 0.466 / 0.410; D3Q13
    // 0.399 / 0.313, 0.717 / 0.627; D3Q19 0.643 / 0.548, 1.146 / 0.981; D3Q27 0.920 / 0.710,
    // 1.647 / 3.591)
    const bool open3d = h->desc.bc != LBM_BC_PERIODIC && h->tab.D == 3 &&
                        !(h->tab.Q > 19 && elem_size(h->desc.storage) == 8);
    // 2-byte storage on boxes of a million cells and more (bound by HBM): the four-cells-per-lane
    // step and its wider accesses (256^3, us per step, GENERIC / DPP, FP16: D3Q13 162 / 147, D3Q19
    // 244 / 231, D3Q27 363 / 332)
    const bool wide = elem_size(h->desc.storage) == 2 && h->N >= ((size_t)1 << 20);
    if (open3d || wide) {
        if (h->nx % 4 == 0) return LBM_VARIANT_DPP;
        if (h->nx % 2 == 0) return LBM_VARIANT_DPP2;
    }
    // everything else (smaller periodic boxes, 4- and 8-byte storage without a multi-step kernel,
    // 1D, large 2D open boxes): one thread per cell.  On small boxes it beats the four-cells-per-lane
    // step for 2-byte storage too (us per step, GENERIC / DPP, FP16: D3Q7 64^3 3.5 / 5.2, 96^3
    // 8.3 / 8.8; D3Q19 64^3 5.8 / 14.7, 96^3 13.5 / 28.6; D2Q9 256^2 3.0 / 3.4)
    return LBM_VARIANT_GENERIC;
}

// Layout of the state buffer as it is now, and the one a fresh state is written in.
inline Layout layout_now(const lbm_lee *h) {
    Layout l{kLayoutPlain, h->nx, h->ny, h->nz};
    if (h->inplace) l.mode = h->phase == 0 ? kLayoutSwapped : kLayoutPushed;
    return l;
}
inline Layout layout_fresh(const lbm_lee *h) {
    Layout l{h->inplace ? kLayoutSwapped : kLayoutPlain, h->nx, h->ny, h->nz};
    return l;
}
// The other ping-pong buffer's rest plane (kept equal to this one's when the step skips it).
inline void *rest_copy_buffer(const lbm_lee *h) { return (h->skip0 && !h->inplace) ? h->buf[h->cur ^ 1] : nullptr; }

// One step launch sequence per velocity set (one translation unit each): advances h by nsteps.
template <class VS>
lbm_status step_lattice(lbm_lee *h, int64_t nsteps, hipStream_t st);

}  // namespace api
}  // namespace lbm
