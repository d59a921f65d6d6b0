// HIP kernels of the LEE lattice Boltzmann scheme for gfx950.
//
// The time step is the fully discrete LBE update (Section "Derivation of the Lattice
// Boltzmann Equation") in pull form: every cell gathers g_i from x - c_i (streaming), takes
// the moments rho', u', theta' (monoatomic / polyatomic FDVM sections), builds the
// equilibrium of the polyatomic ansatz and relaxes with 1/tau.  The collision conserves the
// moments (the equilibrium map is a projection), so moments of the pre- and post-collision
// states agree and the pull form is the paper's push form shifted by one half step.  A state
// set to equilibrium is a fixed point of the collision, so the initial condition g = g^eq
// may be stored as a post-collision state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "codec.hpp"
#include "velsets.hpp"

namespace lbm {

// ------------------------------------------------------------------ constants
// A constant of the collision carried as hi + lo (lo = the rounding residual of hi).  The
// products below use fma(hi, x, lo * x), so a constant enters with ~2^-48 relative error
// in FP32.  With the constant rounded to FP32 alone, the rounding would be the same in
// every cell and every step: the collision would no longer be an exact reflection in the
// 1/f* weighted norm and the error would grow linearly with the step count.
template <typename CT>
struct Kc {
    CT hi, lo;
};

template <bool SPLIT, typename CT>
__device__ __forceinline__ CT mulk(CT x, Kc<CT> k) {
#pragma clang fp contract(off)
    if constexpr (SPLIT)
        return fma(k.hi, x, k.lo * x);
    else
        return k.hi * x;
}

// Only FP32 storage needs the split: FP64 constants are exact to 2^-53, and for the 16-bit
// formats the rounding of every stored value (2^-9 .. 2^-12 relative) dominates the 2^-24
// constant error by orders of magnitude.
template <class ST>
constexpr bool split_constants() {
    return sizeof(typename ST::elem) == 4;
}

// Collision constants in storage units (the raw domain of the storage type in the bulk step
// kernels, ST::dec_raw / enc_raw), for compute type CT, per shell: the populations with
// the same |c_i|^2 (0 rest, 1 axes, 2 edges, 3 corners) share f*_i, beta_i and hence every
// constant below (the host checks this for each table).  With stored value s_i and decoded
// population g_i = dec_i s_i the moments are
//   rho'  = sum_shell dec (sum s_i),      e = sum_shell edec (sum s_i),
//   U     = b u' = sum_shell bu (sum c_i s_i),        bu = b dec / rho0,
//   theta' = gm1_rho0 e - theta0_rho0 rho',
//   A = a1 rho' + a2 theta',  C = c1 rho' + c2 theta',
// and the update s_i <- keep s_i + w (A + |c_i|^2/2 C + c_i.U), keep = 1 - 1/tau and
// w = (1/tau) enc_i f*_i (the equilibrium in storage units).  Every term is linear in the
// per-shell sums, so the host folds the constants (in FP64) into
//   H[to][from]  = w_to (kA dec_from + kA' edec_from + |c_to|^2/2 (kC dec_from + kC' edec_from)),
//   WB[to][from] = w_to bu_from,
// with kA = a1 - a2 theta0_rho0, kA' = a2 gm1_rho0 and kC, kC' likewise from c1, c2, and the
// step computes s_i <- keep s_i + sum_from H[sh_i][from] S_from + c_i . sum_from WB[sh_i][from] J_from
// from the shell sums S and J = sum c_i s_i.
constexpr int kShells = 4;

template <typename CT, int Q>
struct StepCoef {
    Kc<CT> H[kShells][kShells];
    Kc<CT> WB[kShells][kShells];
    Kc<CT> keep;
};

// FP64 constants of the non-hot kernels (init, moments, reductions, import/export).
template <int Q>
struct FieldCoef {
    double f[Q];      // f*_i
    double dec[Q];    // g_i = dec_i s_i
    double enc[Q];    // s_i = enc_i g_i
    double e[Q];      // (|c_i|^2 + beta_i) / 2
    double rho0, theta0, gm1, a1, a2, b, c1, c2;
};

// Is population i the first (from i0 on) of its shell, or with axis >= 0, the first of its
// shell with a nonzero velocity component along that axis?
template <class VS, int i0>
constexpr bool first_of(int i, int axis) {
    for (int j = i0; j < i; ++j)
        if (VS::c2(j) == VS::c2(i) && (axis < 0 || VS::c[j][axis] != 0)) return false;
    return true;
}

template <class VS, bool SKIP0>
constexpr bool has_shell(int sh) {
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i)
        if (VS::c2(i) == sh) return true;
    return false;
}

// fma with a split constant: k t + c with ~2^-48 relative error in the constant.
template <bool SPLIT, typename CT>
__device__ __forceinline__ CT fmak(Kc<CT> k, CT t, CT c) {
#pragma clang fp contract(off)
    if constexpr (SPLIT)
        return fma(k.hi, t, fma(k.lo, t, c));
    else
        return fma(k.hi, t, c);
}

// acc + k x: one fma with a plain constant; with a split one the product is formed first
// (as mulk) and then added, so that the sum sees the same product in both cases.
template <bool SPLIT, typename CT>
__device__ __forceinline__ CT addk(CT acc, CT x, Kc<CT> k) {
#pragma clang fp contract(off)
    if constexpr (SPLIT)
        return acc + mulk<SPLIT>(x, k);
    else
        return fma(k.hi, x, acc);
}

// ------------------------------------------------------------------ collision
// SKIP0: the rest population (index 0) is left out: the host enables this only when the
// equilibrium map leaves it invariant (E_00 = 1, E_0j = E_j0 = 0), in which case the moving
// populations' equilibria do not depend on it either.
// HALF: tau = 1/2 (keep = -1), the paper's second-order choice: s_i <- (relaxed equilibrium)
// - s_i, the same bits as keep s_i + (relaxed equilibrium) with keep = -1.
template <class VS, typename CT, bool SPLIT, bool SKIP0 = false, bool HALF = false>
__device__ __forceinline__ void collide(const StepCoef<CT, VS::Q> &k, CT (&s)[VS::Q]) {
    // No implicit contraction: every fused multiply-add below is written out, so the result
    // does not depend on how the compiler schedules the surrounding kernel (all step variants,
    // the in-place step and the boundary recompute give the same bits for the same inputs).
#pragma clang fp contract(off)
    constexpr int i0 = SKIP0 ? 1 : 0;
    // Sums start from the first term (not from 0 + term, which IEEE arithmetic cannot drop).
    CT sum[kShells] = {}, jx[kShells] = {}, jy[kShells] = {}, jz[kShells] = {};
#pragma unroll
    for (int i = i0; i < VS::Q; ++i) {
        const int sh = VS::c2(i);
        const CT v = s[i];
        if (first_of<VS, i0>(i, -1)) sum[sh] = v; else sum[sh] += v;
        if (VS::cx(i) != 0) {
            const CT sv = VS::cx(i) > 0 ? v : -v;
            if (first_of<VS, i0>(i, 0)) jx[sh] = sv; else jx[sh] += sv;
        }
        if (VS::cy(i) != 0) {
            const CT sv = VS::cy(i) > 0 ? v : -v;
            if (first_of<VS, i0>(i, 1)) jy[sh] = sv; else jy[sh] += sv;
        }
        if (VS::cz(i) != 0) {
            const CT sv = VS::cz(i) > 0 ? v : -v;
            if (first_of<VS, i0>(i, 2)) jz[sh] = sv; else jz[sh] += sv;
        }
    }
    // relaxed equilibrium per target shell: E = H . S, V = WB . J (J only for moving shells)
    CT E[kShells] = {}, Vx[kShells] = {}, Vy[kShells] = {}, Vz[kShells] = {};
#pragma unroll
    for (int to = 0; to < kShells; ++to) {
        if (!has_shell<VS, SKIP0>(to)) continue;
        bool first = true;
#pragma unroll
        for (int from = 0; from < kShells; ++from) {
            if (!has_shell<VS, SKIP0>(from)) continue;
            E[to] = first ? mulk<SPLIT>(sum[from], k.H[to][from]) : addk<SPLIT>(E[to], sum[from], k.H[to][from]);
            first = false;
        }
        if (to == 0) continue;  // the rest velocity carries no momentum term
        bool firstu = true;
#pragma unroll
        for (int from = 1; from < kShells; ++from) {
            if (!has_shell<VS, SKIP0>(from)) continue;
            if (firstu) {
                Vx[to] = mulk<SPLIT>(jx[from], k.WB[to][from]);
                if (VS::D >= 2) Vy[to] = mulk<SPLIT>(jy[from], k.WB[to][from]);
                if (VS::D >= 3) Vz[to] = mulk<SPLIT>(jz[from], k.WB[to][from]);
            } else {
                Vx[to] = addk<SPLIT>(Vx[to], jx[from], k.WB[to][from]);
                if (VS::D >= 2) Vy[to] = addk<SPLIT>(Vy[to], jy[from], k.WB[to][from]);
                if (VS::D >= 3) Vz[to] = addk<SPLIT>(Vz[to], jz[from], k.WB[to][from]);
            }
            firstu = false;
        }
    }
#pragma unroll
    for (int i = i0; i < VS::Q; ++i) {
        const int sh = VS::c2(i);
        CT t = E[sh];
        if (VS::cx(i) > 0) t += Vx[sh];
        if (VS::cx(i) < 0) t -= Vx[sh];
        if (VS::cy(i) > 0) t += Vy[sh];
        if (VS::cy(i) < 0) t -= Vy[sh];
        if (VS::cz(i) > 0) t += Vz[sh];
        if (VS::cz(i) < 0) t -= Vz[sh];
        if constexpr (HALF)  // keep = -1 exactly
            s[i] = t - s[i];
        else
            s[i] = mulk<SPLIT>(s[i], k.keep) + t;
    }
}

__device__ __forceinline__ int wrap_add(int v, int d, int n) {
    v += d;
    if (v < 0) v += n;
    if (v >= n) v -= n;
    return v;
}

// ------------------------------------------------------------------ step: generic variant
// One thread per cell, each population gathered with its own wrapped index.  Any extents.
template <class VS, class ST, bool SKIP0, bool HALF = false>
__global__ __launch_bounds__(256) void step_generic(const typename ST::elem *__restrict__ src,
                                                    typename ST::elem *__restrict__ dst, int nx, int ny, int nz,
                                                    size_t N, StepCoef<typename ST::comp, VS::Q> k) {
    using CT = typename ST::comp;
    const size_t cell = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (cell >= N) return;
    const int x = (int)(cell % (size_t)nx);
    const size_t r = cell / (size_t)nx;
    const int y = (int)(r % (size_t)ny);
    const int z = (int)(r / (size_t)ny);
    CT s[VS::Q];
    s[0] = 0;
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
        const int xs = wrap_add(x, -VS::cx(i), nx);
        const int ys = wrap_add(y, -VS::cy(i), ny);
        const int zs = wrap_add(z, -VS::cz(i), nz);
        s[i] = dec_io<ST, ST::has_raw>(src[(size_t)i * N + ((size_t)zs * ny + ys) * nx + xs]);
    }
    collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(k, s);
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) dst[(size_t)i * N + cell] = enc_io<ST, ST::has_raw>(s[i]);
}

// ------------------------------------------------------------------ step: DPP variant
// DPP controls of whole-wave moves (GFX9 family): lane l receives from lane l-1 (shr/ror)
// or l+1 (shl/rol); the rotations wrap lane 0 <-> lane 63.
enum : int { kDppWaveShl1 = 0x130, kDppWaveRol1 = 0x134, kDppWaveShr1 = 0x138, kDppWaveRor1 = 0x13C };

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Each wave owns a chunk of 64 * VEC consecutive cells of one x-row (VEC cells per lane).
// Rows along y/z are whole-row offsets, so every load and store is an aligned VEC-element
// vector.  A population with c_x = +1 needs the element left of each lane's group: it comes
// from the lane below through a DPP move; c_x = -1 needs the element right of the group from
// the lane above.  FULLROW (nx == 64 * VEC) rotates within the wave, which is exactly the
// periodic wrap; otherwise the first lane and the last active lane load their neighbour
// element directly.  Waves walk the chunks grid-stride (one pass when the grid covers them).
// tune: bit 0 = non-temporal stores, bit 1 = non-temporal loads.
enum : unsigned { kTuneNtStore = 1u, kTuneNtLoad = 2u, kTunePersistent = 4u, kTuneInPlace = 32u };

template <class ST, int VEC>
__device__ __forceinline__ void loadv(const typename ST::elem *p, typename ST::comp (&v)[VEC], bool nt) {
    if constexpr (VEC == 4) {
        load4<ST, ST::has_raw>(p, v, nt);
    } else {
        static_assert(VEC == 2, "VEC is 2 or 4");
        load2<ST, ST::has_raw>(p, v, nt);
    }
}
template <class ST, int VEC>
__device__ __forceinline__ void storev(typename ST::elem *p, const typename ST::comp (&v)[VEC], bool nt) {
    if constexpr (VEC == 4) {
        store4<ST, ST::has_raw>(p, v, nt);
    } else {
        store2<ST, ST::has_raw>(p, v, nt);
    }
}

// The populations of one chunk as loaded (still encoded): one aligned VEC-element vector each.
template <class VS, class ST, int VEC>
struct ChunkRaw {
    typedef typename ST::elem ev __attribute__((ext_vector_type(VEC)));
    ev v[VS::Q];
};

template <class VS, class ST, int VEC, bool SKIP0>
__device__ __forceinline__ void load_chunk(const typename ST::elem *__restrict__ src, int nx, int ny, int nz, size_t N,
                                           unsigned row, int chunk, int lane, bool ntl, ChunkRaw<VS, ST, VEC> &r) {
    using V = typename ChunkRaw<VS, ST, VEC>::ev;
    const int y = (int)(row % (unsigned)ny);
    const int z = (int)(row / (unsigned)ny);
    const int x0 = chunk * (64 * VEC) + lane * VEC;
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
        const int ys = wrap_add(y, -VS::cy(i), ny);
        const int zs = wrap_add(z, -VS::cz(i), nz);
        const typename ST::elem *rowp = src + (size_t)i * N + ((size_t)zs * ny + ys) * (size_t)nx;
        V v = {};
        if (x0 < nx) v = vload(reinterpret_cast<const V *>(rowp + x0), ntl);
        r.v[i] = v;
    }
}

// Row ends of a periodic box: the x-neighbour beyond one end of a row is the cell at the other.
// An open box's bulk step passes its own EDGE whose value() gives what is pulled from beyond an
// x face instead, and whose damp() damps the stored cells of a sponge layer (EDGE::layer, and
// sponge_width > 0).
struct WrapEdge {
    static constexpr bool open = false;
    static constexpr bool layer = false;
};

// Decode a loaded chunk, move the x-neighbours across lanes, collide and store.
template <class VS, class ST, int VEC, bool FULLROW, bool SKIP0, bool HALF, class EDGE = WrapEdge>
__device__ __forceinline__ void finish_chunk(const typename ST::elem *__restrict__ src,
                                             typename ST::elem *__restrict__ dst, int nx, int ny, int nz, size_t N,
                                             unsigned row, int chunk, int lane, bool nts,
                                             const StepCoef<typename ST::comp, VS::Q> &k,
                                             const ChunkRaw<VS, ST, VEC> &r, const EDGE &edge = EDGE{}) {
    using CT = typename ST::comp;
    using E = typename ST::elem;
    constexpr bool RAW = ST::has_raw;
    const int y = (int)(row % (unsigned)ny);
    const int z = (int)(row / (unsigned)ny);
    const int x0 = chunk * (64 * VEC) + lane * VEC;
    const bool active = x0 < nx;
    const bool last = (lane == 63) || (x0 + VEC >= nx);

    CT s[VS::Q][VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) s[0][q] = 0;
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
        CT v[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) v[q] = dec_io<ST, RAW>(r.v[i][q]);
        if (VS::cx(i) == 0) {
#pragma unroll
            for (int q = 0; q < VEC; ++q) s[i][q] = v[q];
        } else {
            const int ys = wrap_add(y, -VS::cy(i), ny);
            const int zs = wrap_add(z, -VS::cz(i), nz);
            const E *rowp = src + (size_t)i * N + ((size_t)zs * ny + ys) * (size_t)nx;
            if (VS::cx(i) > 0) {
                CT prev = FULLROW ? dpp_move<kDppWaveRor1>(v[VEC - 1]) : dpp_move<kDppWaveShr1>(v[VEC - 1]);
                if (!FULLROW && lane == 0 && !(EDGE::open && x0 == 0))
                    prev = dec_io<ST, RAW>(rowp[x0 == 0 ? nx - 1 : x0 - 1]);
                if constexpr (EDGE::open) {
                    if (x0 == 0) prev = edge.template value<VS, ST, RAW>(0, i, ys, zs, v[0]);
                }
                s[i][0] = prev;
#pragma unroll
                for (int q = 1; q < VEC; ++q) s[i][q] = v[q - 1];
            } else {
                CT next = FULLROW ? dpp_move<kDppWaveRol1>(v[0]) : dpp_move<kDppWaveShl1>(v[0]);
                if (!FULLROW && last && active && !(EDGE::open && x0 + VEC >= nx))
                    next = dec_io<ST, RAW>(rowp[x0 + VEC >= nx ? 0 : x0 + VEC]);
                if constexpr (EDGE::open) {
                    if (active && x0 + VEC >= nx) next = edge.template value<VS, ST, RAW>(1, i, ys, zs, v[VEC - 1]);
                }
#pragma unroll
                for (int q = 0; q < VEC - 1; ++q) s[i][q] = v[q + 1];
                s[i][VEC - 1] = next;
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
        CT c[VS::Q];
#pragma unroll
        for (int i = 0; i < VS::Q; ++i) c[i] = s[i][q];
        collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(k, c);
#pragma unroll
        for (int i = 0; i < VS::Q; ++i) s[i][q] = c[i];
    }
    const size_t out = ((size_t)z * ny + y) * (size_t)nx + x0;
    if constexpr (EDGE::open && EDGE::layer) {
        if (edge.sponge_width > 0) {  // a sponge layer: cells within its width of a face are damped
            using V = typename ChunkRaw<VS, ST, VEC>::ev;
            const int dyz = min(min(y, ny - 1 - y), min(z, nz - 1 - z));
#pragma unroll
            for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
                V c;
#pragma unroll
                for (int q = 0; q < VEC; ++q) {
                    const E e = enc_io<ST, RAW>(s[i][q]);
                    const int d = min(dyz, min(x0 + q, nx - 1 - x0 - q));
                    c[q] = d < edge.sponge_width ? edge.template damp<ST>(e, d) : e;
                }
                vstore(reinterpret_cast<V *>(dst + (size_t)i * N + out), c, nts);
            }
            return;
        }
    }
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) storev<ST, VEC>(dst + (size_t)i * N + out, s[i], nts);
}

// Each wave owns chunks wave, wave + G, wave + 2G, ... (G = waves in the grid).  Without the
// persistent tuning the grid covers every chunk once.  With it the grid is sized to the resident
// wave slots and every wave loads its next chunk before it finishes the current one, so its
// loads stay in flight across the collision and the waves end together.
template <class VS, class ST, int VEC, bool FULLROW, bool SKIP0, bool HALF = false>
__global__ __launch_bounds__(256) void step_dpp(const typename ST::elem *__restrict__ src,
                                                typename ST::elem *__restrict__ dst, int nx, int ny, int nz,
                                                size_t N, int chunks_per_row, unsigned total_waves, unsigned tune,
                                                StepCoef<typename ST::comp, VS::Q> k) {
    const int lane = threadIdx.x & 63;
    const unsigned wid = (unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool ntl = (tune & kTuneNtLoad) != 0, nts = (tune & kTuneNtStore) != 0;
    const unsigned G = gridDim.x * 4u;
    unsigned wave = blockIdx.x * 4u + wid;
    if (wave >= total_waves) return;
    ChunkRaw<VS, ST, VEC> cur, nxt;
    load_chunk<VS, ST, VEC, SKIP0>(src, nx, ny, nz, N, wave / (unsigned)chunks_per_row,
                                   (int)(wave % (unsigned)chunks_per_row), lane, ntl, cur);
    for (;;) {
        const unsigned wn = wave + G;
        const bool more = wn < total_waves;  // uniform across the wave
        if (more)
            load_chunk<VS, ST, VEC, SKIP0>(src, nx, ny, nz, N, wn / (unsigned)chunks_per_row,
                                           (int)(wn % (unsigned)chunks_per_row), lane, ntl, nxt);
        finish_chunk<VS, ST, VEC, FULLROW, SKIP0, HALF>(src, dst, nx, ny, nz, N, wave / (unsigned)chunks_per_row,
                                                        (int)(wave % (unsigned)chunks_per_row), lane, nts, k, cur);
        if (!more) break;
        cur = nxt;
        wave = wn;
    }
}

// ------------------------------------------------------------------ step: LDS-staged variant
// One thread per cell; a block owns 256 consecutive cells of one x-row.  Populations with
// c_x = 0 are loaded directly (aligned, coalesced).  For c_x != 0 the block stages its own
// 256 source cells plus one halo cell on each side (periodic wrap at the row ends) in LDS with
// aligned loads, and every thread reads its x-shifted value from LDS.
template <class VS>
constexpr int x_moving_count() {
    int n = 0;
    for (int i = 0; i < VS::Q; ++i) n += VS::c[i][0] != 0 ? 1 : 0;
    return n;
}

template <class VS, class ST, bool SKIP0, bool HALF = false>
__global__ __launch_bounds__(256) void step_lds(const typename ST::elem *__restrict__ src,
                                                typename ST::elem *__restrict__ dst, int nx, int ny, int nz,
                                                size_t N, int chunks_per_row, StepCoef<typename ST::comp, VS::Q> k) {
    using CT = typename ST::comp;
    using E = typename ST::elem;
    constexpr int NXM = x_moving_count<VS>() > 0 ? x_moving_count<VS>() : 1;
    __shared__ CT stage[NXM][258];
    const unsigned blk = blockIdx.x;
    const unsigned row = blk / (unsigned)chunks_per_row;
    const int chunk = (int)(blk - row * (unsigned)chunks_per_row);
    const int y = (int)(row % (unsigned)ny);
    const int z = (int)(row / (unsigned)ny);
    const int t = threadIdx.x;
    const int x0 = chunk * 256;
    const int x = x0 + t;
    const bool active = x < nx;
    const int width = min(256, nx - x0);  // cells of this chunk

    CT s[VS::Q];
    s[0] = 0;
    int m = 0;
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
        const int ys = wrap_add(y, -VS::cy(i), ny);
        const int zs = wrap_add(z, -VS::cz(i), nz);
        const E *rowp = src + (size_t)i * N + ((size_t)zs * ny + ys) * (size_t)nx;
        if (VS::cx(i) == 0) {
            s[i] = active ? dec_io<ST, ST::has_raw>(rowp[x]) : (CT)0;
        } else {
            if (active) stage[m][t + 1] = dec_io<ST, ST::has_raw>(rowp[x]);
            if (t == 0) stage[m][0] = dec_io<ST, ST::has_raw>(rowp[x0 == 0 ? nx - 1 : x0 - 1]);
            if (t == 1) stage[m][width + 1] = dec_io<ST, ST::has_raw>(rowp[x0 + width >= nx ? 0 : x0 + width]);
            ++m;
        }
    }
    __syncthreads();
    m = 0;
#pragma unroll
    for (int i = 0; i < VS::Q; ++i) {
        if (VS::cx(i) != 0) {
            s[i] = stage[m][t + 1 - VS::cx(i)];
            ++m;
        }
    }
    if (!active) return;
    collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(k, s);
    const size_t cell = ((size_t)z * ny + y) * (size_t)nx + x;
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) dst[(size_t)i * N + cell] = enc_io<ST, ST::has_raw>(s[i]);
}

// ------------------------------------------------------------------ in-place streaming
// One buffer instead of two (the "AA" pattern of in-place streaming).  The buffer holds the
// post-collision state g*(t) in one of two layouts, alternating step by step:
//   swapped (S): g*_i(x) in slot opposite(i) of cell x;
//   pushed  (P): g*_i(x) in slot i of cell x + c_i (the value cell x + c_i pulls next).
// From P a cell reads its incoming values from its own slots, collides, and writes S into the
// same slots; from S it reads slot opposite(i) of x - c_i and writes slot i of x + c_i, which is
// the same set of locations.  Either way every cell reads and writes only its own set, so the
// update is race-free in place.  The rest population (c = 0) never moves.
template <class VS>
__host__ __device__ constexpr int opposite(int i) {
    for (int j = 0; j < VS::Q; ++j)
        if (VS::c[j][0] == -VS::c[i][0] && VS::c[j][1] == -VS::c[i][1] && VS::c[j][2] == -VS::c[i][2]) return j;
    return -1;
}

template <class VS>
constexpr bool every_velocity_has_opposite() {
    for (int i = 0; i < VS::Q; ++i)
        if (opposite<VS>(i) < 0) return false;
    return true;
}

enum : int { kLayoutPlain = 0, kLayoutSwapped = 1, kLayoutPushed = 2 };

// Where population i of cell (x, y, z) lives in a state buffer of the given layout.
struct Layout {
    int mode;
    int nx, ny, nz;
};

template <class VS>
__device__ __forceinline__ size_t pop_index(const Layout &L, int i, size_t N, size_t cell, int x, int y, int z) {
    if (L.mode == kLayoutSwapped) return (size_t)opposite<VS>(i) * N + cell;
    if (L.mode == kLayoutPushed) {
        const int xs = wrap_add(x, VS::cx(i), L.nx);
        const int ys = wrap_add(y, VS::cy(i), L.ny);
        const int zs = wrap_add(z, VS::cz(i), L.nz);
        return (size_t)i * N + ((size_t)zs * L.ny + ys) * L.nx + xs;
    }
    return (size_t)i * N + cell;
}
template <class VS>
__device__ __forceinline__ size_t pop_index(const Layout &L, int i, size_t N, size_t cell) {
    if (L.mode != kLayoutPushed) return pop_index<VS>(L, i, N, cell, 0, 0, 0);
    const int x = (int)(cell % (size_t)L.nx);
    const size_t r = cell / (size_t)L.nx;
    return pop_index<VS>(L, i, N, cell, x, (int)(r % (size_t)L.ny), (int)(r / (size_t)L.ny));
}

// One in-place step: FROM_S = the buffer holds layout S (and leaves P), else P -> S.
template <class VS, class ST, bool SKIP0, bool HALF, bool FROM_S>
__global__ __launch_bounds__(256) void step_inplace(typename ST::elem *__restrict__ A, int nx, int ny, int nz, size_t N,
                                                    StepCoef<typename ST::comp, VS::Q> k) {
    static_assert(every_velocity_has_opposite<VS>(), "in-place streaming needs a symmetric velocity set");
    using CT = typename ST::comp;
    const size_t cell = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (cell >= N) return;
    const int x = (int)(cell % (size_t)nx);
    const size_t r = cell / (size_t)nx;
    const int y = (int)(r % (size_t)ny);
    const int z = (int)(r / (size_t)ny);
    CT s[VS::Q];
    s[0] = 0;
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
        size_t at = (size_t)i * N + cell;
        if (FROM_S) {
            const int xs = wrap_add(x, -VS::cx(i), nx);
            const int ys = wrap_add(y, -VS::cy(i), ny);
            const int zs = wrap_add(z, -VS::cz(i), nz);
            at = (size_t)opposite<VS>(i) * N + ((size_t)zs * ny + ys) * nx + xs;
        }
        s[i] = dec_io<ST, ST::has_raw>(A[at]);
    }
    collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(k, s);
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
        size_t at = (size_t)opposite<VS>(i) * N + cell;
        if (FROM_S) {
            const int xs = wrap_add(x, VS::cx(i), nx);
            const int ys = wrap_add(y, VS::cy(i), ny);
            const int zs = wrap_add(z, VS::cz(i), nz);
            at = (size_t)i * N + ((size_t)zs * ny + ys) * nx + xs;
        }
        A[at] = enc_io<ST, ST::has_raw>(s[i]);
    }
}

// ------------------------------------------------------------------ initial state
// g_i(0, x) = g_i^eq(rho'(x), u'(x), theta'(x)) in FP64, then encoded to storage.
template <class VS, class ST>
__global__ __launch_bounds__(256) void init_equilibrium(const double *__restrict__ rho, const double *__restrict__ u,
                                                        const double *__restrict__ theta,
                                                        typename ST::elem *__restrict__ dst,
                                                        typename ST::elem *__restrict__ rest_copy, size_t N,
                                                        FieldCoef<VS::Q> k, Layout lay) {
    const size_t cell = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (cell >= N) return;
    const double r = rho[cell], th = theta[cell];
    const double ux = u[cell];
    const double uy = VS::D >= 2 ? u[N + cell] : 0.0;
    const double uz = VS::D >= 3 ? u[2 * N + cell] : 0.0;
    const double A = k.a1 * r + k.a2 * th;
    const double C = k.c1 * r + k.c2 * th;
#pragma unroll
    for (int i = 0; i < VS::Q; ++i) {
        const double cu = VS::cx(i) * ux + VS::cy(i) * uy + VS::cz(i) * uz;
        const double geq = k.f[i] * (A + k.b * cu + 0.5 * VS::c2(i) * C);
        const typename ST::elem v = ST::enc_d(k.enc[i] * geq);
        dst[pop_index<VS>(lay, i, N, cell)] = v;
        if (i == 0 && rest_copy) rest_copy[cell] = v;  // the other buffer's rest plane
    }
}

// Equilibrium of fields given on a sub-box (n_sub cells at origin o), zero elsewhere.
template <class VS, class ST>
__global__ __launch_bounds__(256) void init_region(const double *__restrict__ rho, const double *__restrict__ u,
                                                   const double *__restrict__ theta,
                                                   typename ST::elem *__restrict__ dst,
                                                   typename ST::elem *__restrict__ rest_copy, int nx, int ny, size_t N,
                                                   int ox, int oy, int oz, int sx, int sy, int sz,
                                                   FieldCoef<VS::Q> k, Layout lay) {
    const size_t cell = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (cell >= N) return;
    const int x = (int)(cell % nx) - ox;
    const size_t r = cell / nx;
    const int y = (int)(r % ny) - oy, z = (int)(r / ny) - oz;
    double rr = 0, th = 0, ux = 0, uy = 0, uz = 0;
    if (x >= 0 && x < sx && y >= 0 && y < sy && z >= 0 && z < sz) {
        const size_t Ns = (size_t)sx * sy * sz;
        const size_t sc = ((size_t)z * sy + y) * sx + x;
        rr = rho[sc];
        th = theta[sc];
        ux = u[sc];
        if (VS::D >= 2) uy = u[Ns + sc];
        if (VS::D >= 3) uz = u[2 * Ns + sc];
    }
    const double A = k.a1 * rr + k.a2 * th;
    const double C = k.c1 * rr + k.c2 * th;
#pragma unroll
    for (int i = 0; i < VS::Q; ++i) {
        const double cu = VS::cx(i) * ux + VS::cy(i) * uy + VS::cz(i) * uz;
        const double geq = k.f[i] * (A + k.b * cu + 0.5 * VS::c2(i) * C);
        const typename ST::elem v = ST::enc_d(k.enc[i] * geq);
        dst[pop_index<VS>(lay, i, N, cell)] = v;
        if (i == 0 && rest_copy) rest_copy[cell] = v;
    }
}

// ------------------------------------------------------------------ block reductions (FP64)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Reduce NV values per thread over a 256-thread block; thread 0 gets the result.  Fixed
// order (lane tree, then waves 0..3), so a launch with a fixed grid is deterministic.
// IS_MAX[j] selects max instead of sum for value j.
template <int NV>
__device__ void block_reduce(double (&v)[NV], const bool (&is_max)[NV]) {
    __shared__ double part[4][NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = is_max[j] ? wave_max(v[j]) : wave_sum(v[j]);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) part[wv][j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double a = part[0][j];
            for (int w = 1; w < 4; ++w) a = is_max[j] ? fmax(a, part[w][j]) : a + part[w][j];
            v[j] = a;
        }
    }
}

// Second pass: one block folds `nblk` partial rows (NV doubles each) in a fixed order.
template <int NV>
__global__ __launch_bounds__(256) void reduce_partials(const double *__restrict__ part, int nblk,
                                                       double *__restrict__ out, unsigned max_mask) {
    double v[NV];
    bool is_max[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        is_max[j] = (max_mask >> j) & 1u;
        v[j] = 0.0;
    }
    for (int b = threadIdx.x; b < nblk; b += 256)
#pragma unroll
        for (int j = 0; j < NV; ++j) v[j] = is_max[j] ? fmax(v[j], part[(size_t)b * NV + j]) : v[j] + part[(size_t)b * NV + j];
    block_reduce<NV>(v, is_max);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) out[j] = v[j];
}

// Weighted and plain energy of the current state: per-block partials of
// sum g^2 / f* and sum g^2, FP64, grid-stride over cells.
template <class VS, class ST>
__global__ __launch_bounds__(256) void energy_partials(const typename ST::elem *__restrict__ src, size_t N,
                                                       FieldCoef<VS::Q> k, double *__restrict__ part) {
    double v[2] = {0.0, 0.0};
    const bool is_max[2] = {false, false};
    for (size_t cell = (size_t)blockIdx.x * 256u + threadIdx.x; cell < N; cell += (size_t)gridDim.x * 256u) {
#pragma unroll
        for (int i = 0; i < VS::Q; ++i) {
            const double g = k.dec[i] * (double)ST::dec(src[(size_t)i * N + cell]);
            v[0] += g * g / k.f[i];
            v[1] += g * g;
        }
    }
    block_reduce<2>(v, is_max);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v[0];
        part[2 * blockIdx.x + 1] = v[1];
    }
}

// FP64 moments of one cell of the current state.
template <class VS, class ST>
__device__ __forceinline__ void cell_moments(const typename ST::elem *__restrict__ src, size_t N, size_t cell,
                                             const FieldCoef<VS::Q> &k, double &rho, double (&u)[3], double &theta,
                                             double &p, const Layout &lay) {
    double r = 0, jx = 0, jy = 0, jz = 0, e = 0;
#pragma unroll
    for (int i = 0; i < VS::Q; ++i) {
        const double g = k.dec[i] * (double)ST::dec(src[pop_index<VS>(lay, i, N, cell)]);
        r += g;
        jx += VS::cx(i) * g;
        jy += VS::cy(i) * g;
        jz += VS::cz(i) * g;
        e += k.e[i] * g;
    }
    rho = r;
    u[0] = jx / k.rho0;
    u[1] = jy / k.rho0;
    u[2] = jz / k.rho0;
    theta = (k.gm1 * e - k.theta0 * r) / k.rho0;
    p = k.rho0 * theta + k.theta0 * r;
}

template <class VS, class ST, typename OT>
__global__ __launch_bounds__(256) void moments_kernel(const typename ST::elem *__restrict__ src, size_t N,
                                                      FieldCoef<VS::Q> k, OT *__restrict__ p, OT *__restrict__ u,
                                                      OT *__restrict__ rho, OT *__restrict__ theta, Layout lay) {
    const size_t cell = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (cell >= N) return;
    double r, uu[3], th, pp;
    cell_moments<VS, ST>(src, N, cell, k, r, uu, th, pp, lay);
    if (p) p[cell] = (OT)pp;
    if (rho) rho[cell] = (OT)r;
    if (theta) theta[cell] = (OT)th;
    if (u)
#pragma unroll
        for (int a = 0; a < VS::D; ++a) u[(size_t)a * N + cell] = (OT)uu[a];
}

// Moments of the cells of a sub-box (n_sub cells at origin o); outputs are sub-box arrays.
template <class VS, class ST, typename OT>
__global__ __launch_bounds__(256) void moments_region_kernel(const typename ST::elem *__restrict__ src, size_t N,
                                                             int nx, int ny, int ox, int oy, int oz, int sx, int sy,
                                                             int sz, FieldCoef<VS::Q> k, OT *__restrict__ p,
                                                             OT *__restrict__ u, OT *__restrict__ rho,
                                                             OT *__restrict__ theta, Layout lay) {
    const size_t Ns = (size_t)sx * sy * sz;
    const size_t sc = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (sc >= Ns) return;
    const int x = (int)(sc % sx);
    const size_t r = sc / sx;
    const int y = (int)(r % sy), z = (int)(r / sy);
    const size_t cell = ((size_t)(z + oz) * ny + (y + oy)) * nx + (x + ox);
    double rr, uu[3], th, pp;
    cell_moments<VS, ST>(src, N, cell, k, rr, uu, th, pp, lay);
    if (p) p[sc] = (OT)pp;
    if (rho) rho[sc] = (OT)rr;
    if (theta) theta[sc] = (OT)th;
    if (u)
#pragma unroll
        for (int a = 0; a < VS::D; ++a) u[(size_t)a * Ns + sc] = (OT)uu[a];
}

// Error against reference fields: per-block partials of
// { sum dp^2, sum p_ref^2, max |dp|, sum |du|^2, sum |u_ref|^2, max |du_a| }.
template <class VS, class ST>
__global__ __launch_bounds__(256) void error_partials(const typename ST::elem *__restrict__ src, size_t N,
                                                      FieldCoef<VS::Q> k, const double *__restrict__ ref_p,
                                                      const double *__restrict__ ref_u, double *__restrict__ part,
                                                      Layout lay) {
    double v[6] = {0, 0, 0, 0, 0, 0};
    const bool is_max[6] = {false, false, true, false, false, true};
    for (size_t cell = (size_t)blockIdx.x * 256u + threadIdx.x; cell < N; cell += (size_t)gridDim.x * 256u) {
        double r, uu[3], th, pp;
        cell_moments<VS, ST>(src, N, cell, k, r, uu, th, pp, lay);
        const double dp = pp - ref_p[cell];
        v[0] += dp * dp;
        v[1] += ref_p[cell] * ref_p[cell];
        v[2] = fmax(v[2], fabs(dp));
        if (ref_u) {
#pragma unroll
            for (int a = 0; a < VS::D; ++a) {
                const double ur = ref_u[(size_t)a * N + cell];
                const double du = uu[a] - ur;
                v[3] += du * du;
                v[4] += ur * ur;
                v[5] = fmax(v[5], fabs(du));
            }
        }
    }
    block_reduce<6>(v, is_max);
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < 6; ++j) part[6 * blockIdx.x + j] = v[j];
}

// Max over cells and populations of |g^eq_i / f*_i| of the initial fields (storage scale).
template <class VS>
__global__ __launch_bounds__(256) void scale_partials(const double *__restrict__ rho, const double *__restrict__ u,
                                                      const double *__restrict__ theta, size_t N, FieldCoef<VS::Q> k,
                                                      double *__restrict__ part) {
    double v[1] = {0.0};
    const bool is_max[1] = {true};
    for (size_t cell = (size_t)blockIdx.x * 256u + threadIdx.x; cell < N; cell += (size_t)gridDim.x * 256u) {
        const double r = rho[cell], th = theta[cell];
        const double ux = u[cell];
        const double uy = VS::D >= 2 ? u[N + cell] : 0.0;
        const double uz = VS::D >= 3 ? u[2 * N + cell] : 0.0;
        const double A = k.a1 * r + k.a2 * th, C = k.c1 * r + k.c2 * th;
#pragma unroll
        for (int i = 0; i < VS::Q; ++i) {
            const double cu = VS::cx(i) * ux + VS::cy(i) * uy + VS::cz(i) * uz;
            v[0] = fmax(v[0], fabs(A + k.b * cu + 0.5 * VS::c2(i) * C));
        }
    }
    block_reduce<1>(v, is_max);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// ------------------------------------------------------------------ import / export
template <class VS, class ST>
__global__ __launch_bounds__(256) void export_f64(const typename ST::elem *__restrict__ src, size_t N,
                                                  FieldCoef<VS::Q> k, double *__restrict__ g, Layout lay) {
    const size_t idx = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (idx >= (size_t)VS::Q * N) return;
    const int i = (int)(idx / N);
    double d = k.dec[0];
#pragma unroll
    for (int j = 1; j < VS::Q; ++j)
        if (j == i) d = k.dec[j];
    g[idx] = d * (double)ST::dec(src[pop_index<VS>(lay, i, N, idx - (size_t)i * N)]);
}

template <class VS, class ST>
__global__ __launch_bounds__(256) void import_f64(const double *__restrict__ g, size_t N, FieldCoef<VS::Q> k,
                                                  typename ST::elem *__restrict__ dst,
                                                  typename ST::elem *__restrict__ rest_copy, Layout lay) {
    const size_t idx = (size_t)blockIdx.x * 256u + threadIdx.x;
    if (idx >= (size_t)VS::Q * N) return;
    const int i = (int)(idx / N);
    double e = k.enc[0];
#pragma unroll
    for (int j = 1; j < VS::Q; ++j)
        if (j == i) e = k.enc[j];
    const typename ST::elem v = ST::enc_d(e * g[idx]);
    dst[pop_index<VS>(lay, i, N, idx - (size_t)i * N)] = v;
    if (i == 0 && rest_copy) rest_copy[idx] = v;
}

// ------------------------------------------------------------------ plain copy (calibration)
[[maybe_unused]] static __global__ __launch_bounds__(256) void copy16(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst, size_t n16) {
    for (size_t i = (size_t)blockIdx.x * 256u + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256u) dst[i] = src[i];
}

}  // namespace lbm
