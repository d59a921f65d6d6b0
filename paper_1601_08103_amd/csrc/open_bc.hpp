// Open (non-periodic) boundaries of the box.  Not in the paper, which treats periodic
// domains only and names boundary conditions as future work.
//
// One step on an open box: the bulk step kernel runs on every cell as if periodic, then the
// shell kernel recomputes every boundary cell (a cell whose pull crosses a face), taking the
// streamed value of a population whose source s = x - c_i lies outside from the closure:
//   ZERO / SPONGE : 0 (exterior at rest);
//   COPY          : the value at clamp(s) (zero normal gradient);
//   MLP           : the learned prediction for the face node clamp(s) (mean over every face
//                   the source lies beyond, for edge and corner sources).
// SPONGE then damps the new post-collision state by 1 - sigma_max ((W - d) / W)^2 at distance
// d < W from the nearest face.
//
// Face f = 2a + side (axis a, side 0 = low, 1 = high).  A signed axis permutation maps the
// face's outward normal to -x; perm[f][j] is the population whose velocity maps to canonical
// velocity j, and the populations entering through the face are the canonical ones with
// c_x = +1 (rank r in canonical order).  Nodes of face f are its cells, numbered over the two
// in-face axes (ascending, the lower one fastest); global node ids run face after face.
#pragma once

#include <hip/hip_runtime.h>

#include "codec.hpp"
#include "kernels.hpp"
#include "nrbc.hpp"
#include "velsets.hpp"

namespace lbm {

enum : int { kBcPeriodic = 0, kBcZero = 1, kBcCopy = 2, kBcSponge = 3, kBcMlp = 4 };

template <int Q>
struct FaceTab {
    int nfaces;
    signed char perm[6][Q];  // canonical j -> face population
    signed char rank[6][Q];  // face population -> entering rank, -1 if not entering
    long long node_off[7];   // first global node of each face; node_off[nfaces] = total
    int n[3];
    int D;
};

// In-face axes of axis a (ascending); -1 when absent.
__host__ __device__ inline void infaces(int a, int D, int &t1, int &t2) {
    t1 = t2 = -1;
    for (int b = 0; b < D; ++b)
        if (b != a) {
            if (t1 < 0)
                t1 = b;
            else
                t2 = b;
        }
}

template <int Q>
__device__ inline long long node_index(const FaceTab<Q> &ft, int f, const int (&p)[3]) {
    int t1, t2;
    infaces(f >> 1, ft.D, t1, t2);
    long long nd = 0;
    if (t1 >= 0) nd = p[t1];
    if (t2 >= 0) nd += (long long)ft.n[t1] * p[t2];
    return ft.node_off[f] + nd;
}

// Face and cell of global node g.  Offsets and extents are read at fixed indices (kernel
// arguments stay in scalar registers) and selected, so no lookup waits on a memory load.
template <int Q>
__device__ inline int node_cell(const FaceTab<Q> &ft, long long g, int (&p)[3]) {
    const int n[3] = {ft.n[0], ft.n[1], ft.n[2]};
    int f = 0;
    long long lo = 0;  // node_off[0] = 0
#pragma unroll
    for (int k = 1; k < 6; ++k) {
        const long long o = ft.node_off[k];
        if (k < ft.nfaces && g >= o) {  // offsets increase: the last face starting at or before g
            f = k;
            lo = o;
        }
    }
    long long nd = g - lo;
    const int a = f >> 1;
    int t1, t2;
    infaces(a, ft.D, t1, t2);
    auto ext = [&](int b) { return b == 0 ? n[0] : (b == 1 ? n[1] : n[2]); };
    p[0] = p[1] = p[2] = 0;
    int q1 = 0, q2 = 0;
    if (t1 >= 0) {
        const int m = ext(t1);
        if (nd <= 0x7fffffffLL) {  // 32-bit division when it fits (64-bit division is emulated)
            const unsigned u = (unsigned)nd, um = (unsigned)m;
            q1 = (int)(u % um);
            nd = u / um;
        } else {
            q1 = (int)(nd % m);
            nd /= m;
        }
    }
    if (t2 >= 0) q2 = (int)nd;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (b == t1) p[b] = q1;
        if (b == t2) p[b] = q2;
        if (b == a) p[b] = (f & 1) ? ext(a) - 1 : 0;
    }
    return f;
}

// ------------------------------------------------------------------ sponge damping
// Damping factor at distance d < width from the nearest face, and a stored value damped by it
// (decoded, scaled, encoded again).
template <class CT>
__device__ inline CT sponge_factor(int d, int width, double sigma_max) {
    const CT w = (CT)(width - d) / (CT)width;
    return (CT)1 - (CT)sigma_max * w * w;
}
template <class ST>
__device__ inline typename ST::elem sponge_damp(typename ST::elem e, typename ST::comp fac) {
    return ST::enc(ST::dec(e) * fac);
}

// ------------------------------------------------------------------ shell recompute
// Streamed values of boundary cell x, in two passes: shell_inside takes every source inside the
// box (every source with COPY, clamped) from the state and leaves 0 for the others (ZERO,
// SPONGE); shell_outside then fills, with MLP, each outside source i with the mean over the
// faces fb it lies beyond of the prediction GH(fb, clamp(s), i) (the face node's value for the
// rank population i enters with), times GH.enc(i) (physical to stored units).
template <class VS, class ST, bool SKIP0>
__device__ inline void shell_inside(const typename ST::elem *__restrict__ src, size_t N, int closure,
                                    const int (&x)[3], const FaceTab<VS::Q> &ft, typename ST::comp (&s)[VS::Q]) {
    using CT = typename ST::comp;
    s[0] = 0;
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
        const int c[3] = {VS::cx(i), VS::cy(i), VS::cz(i)};
        int cl[3];
        bool inside = true;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int sp = x[b] - c[b];
            cl[b] = min(max(sp, 0), ft.n[b] - 1);
            inside = inside && sp == cl[b];
        }
        const size_t scell = ((size_t)cl[2] * ft.n[1] + cl[1]) * ft.n[0] + cl[0];
        s[i] = (inside || closure == kBcCopy) ? (CT)ST::dec(src[(size_t)i * N + scell]) : (CT)0;
    }
}

template <class VS, class ST, bool SKIP0, class GH>
__device__ inline void shell_outside(const int (&x)[3], const int (&n)[3], typename ST::comp (&s)[VS::Q], GH ghost_at) {
    using CT = typename ST::comp;
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
        const int c[3] = {VS::cx(i), VS::cy(i), VS::cz(i)};
        int sp[3], cl[3];
        bool inside = true;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            sp[b] = x[b] - c[b];
            cl[b] = min(max(sp[b], 0), n[b] - 1);
            inside = inside && sp[b] == cl[b];
        }
        if (inside) continue;
        float acc = 0.0f;
        int cnt = 0;
#pragma unroll
        for (int b = 0; b < VS::D; ++b) {
            if (sp[b] != cl[b]) {
                const int fb = 2 * b + (sp[b] > cl[b] ? 1 : 0);
                acc += ghost_at(fb, cl, i);
                ++cnt;
            }
        }
        s[i] = (CT)(acc / (float)cnt) * ghost_at.enc(i);
    }
}

// Grid (x blocks, one y block per face).  bulk_x: the bulk step (step_dpp_open) has already
// computed the x faces' cells of every row that lies on no y or z face; the grid then covers the
// y and z faces only (blockIdx.y + 2), which own their cells on the x faces.  sponge_width > 0
// (only with bulk_x): the cells stored are damped as the sponge kernel would damp them.
template <class VS, class ST, bool SKIP0, bool HALF = false>
__global__ __launch_bounds__(256) void shell_kernel(const typename ST::elem *__restrict__ src,
                                                    typename ST::elem *__restrict__ dst, size_t N, int closure,
                                                    const float *__restrict__ ghost, FaceTab<VS::Q> ft,
                                                    StepCoef<typename ST::comp, VS::Q> k, FieldCoef<VS::Q> fk,
                                                    int bulk_x, int sponge_width, double sponge_sigma) {
    using CT = typename ST::comp;
    const int f = (int)blockIdx.y + (bulk_x ? 2 : 0);
    const int a = f >> 1, side = f & 1;
    int t1, t2;
    infaces(a, VS::D, t1, t2);
    // cells of this face not already owned by a face of a lower axis (with bulk_x the x faces own
    // none: their rows off the other faces are the bulk step's)
    const int lo1 = (t1 >= 0 && t1 < a && !(bulk_x && t1 == 0)) ? 1 : 0;
    const int lo2 = (t2 >= 0 && t2 < a && !(bulk_x && t2 == 0)) ? 1 : 0;
    const int n1 = t1 >= 0 ? ft.n[t1] - 2 * lo1 : 1, n2 = t2 >= 0 ? ft.n[t2] - 2 * lo2 : 1;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)n1 * n2) return;
    int x[3] = {0, 0, 0};
    if (t <= 0x7fffffffLL) {  // 32-bit division when it fits
        if (t1 >= 0) x[t1] = (int)((unsigned)t % (unsigned)n1) + lo1;
        if (t2 >= 0) x[t2] = (int)((unsigned)t / (unsigned)n1) + lo2;
    } else {
        if (t1 >= 0) x[t1] = (int)(t % n1) + lo1;
        if (t2 >= 0) x[t2] = (int)(t / n1) + lo2;
    }
    x[a] = side ? ft.n[a] - 1 : 0;
    const size_t cell = ((size_t)x[2] * ft.n[1] + x[1]) * ft.n[0] + x[0];
    constexpr int K = entering_count<VS>();

    CT s[VS::Q];
    shell_inside<VS, ST, SKIP0>(src, N, closure, x, ft, s);
    if (closure == kBcMlp) {
        struct {
            const float *ghost;
            const FaceTab<VS::Q> &ft;
            const FieldCoef<VS::Q> &fk;
            __device__ float operator()(int fb, const int (&cl)[3], int i) const {
                const int r = ft.rank[fb][i];
                return ghost[node_index(ft, fb, cl) * K + (r < 0 ? 0 : r)];
            }
            __device__ CT enc(int i) const { return (CT)fk.enc[i]; }
        } gh{ghost, ft, fk};
        const int n[3] = {ft.n[0], ft.n[1], ft.n[2]};
        shell_outside<VS, ST, SKIP0>(x, n, s, gh);
    }
    collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(k, s);
    if (sponge_width > 0) {  // with bulk_x, a sponge layer: face cells lie at distance 0
        const CT fac = sponge_factor<CT>(0, sponge_width, sponge_sigma);
#pragma unroll
        for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) dst[(size_t)i * N + cell] = sponge_damp<ST>(ST::enc(s[i]), fac);
        return;
    }
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) dst[(size_t)i * N + cell] = ST::enc(s[i]);
}

// ------------------------------------------------------------------ bulk step of an open box
// The one-step DPP bulk kernel with the x faces closed in the bulk step itself: where a row's
// end cell pulls from beyond an x face (population i with c_x = +1 at x = 0, c_x = -1 at
// x = nx - 1), it takes the closure's value there instead of the other end of the row: 0 for
// ZERO and SPONGE, the row's end cell itself for COPY (the clamped source), and for MLP the face
// node's prediction in stored units, the value shell_outside forms for a source beyond one face.
// Rows on a y or z face pull from beyond those faces too; the shell kernel recomputes them.  So
// the x faces, whose cells are strided in memory, cost no second pass.  A sponge layer
// (sponge_width > 0) is damped as each cell is stored, as the sponge kernel damps a stored value;
// the shell kernel damps the face cells it recomputes, so no sponge pass is needed either.
template <int Q, bool LAYER>
struct OpenEdge {
    static constexpr bool open = true;
    static constexpr bool layer = LAYER;  // compiled with the damping path (kept out of other boxes' code)
    int closure;
    const float *ghost;
    const FaceTab<Q> &ft;
    const FieldCoef<Q> &fk;
    int sponge_width;
    double sponge_sigma;
    template <class ST>
    __device__ typename ST::elem damp(typename ST::elem e, int d) const {
        return sponge_damp<ST>(e, sponge_factor<typename ST::comp>(d, sponge_width, sponge_sigma));
    }
    // side 0: the low x face (sources at x = -1), 1: the high one; (ys, zs) the source row
    template <class VS, class ST, bool RAW>
    __device__ typename ST::comp value(int side, int i, int ys, int zs, typename ST::comp own) const {
        using CT = typename ST::comp;
        if (closure == kBcCopy) return own;
        if (closure != kBcMlp) return (CT)0;
        const int p[3] = {side ? ft.n[0] - 1 : 0, ys, zs};
        const int r = ft.rank[side][i];
        CT v = (CT)ghost[node_index(ft, side, p) * entering_count<VS>() + (r < 0 ? 0 : r)] * (CT)fk.enc[i];
        if constexpr (RAW) v *= (CT)ST::raw_unit;
        return v;
    }
};

// Same chunk walk as step_dpp (including the persistent tuning).  LAYER: with a sponge layer.
template <class VS, class ST, int VEC, bool FULLROW, bool SKIP0, bool HALF, bool LAYER>
__global__ __launch_bounds__(256) void step_dpp_open(const typename ST::elem *__restrict__ src,
                                                     typename ST::elem *__restrict__ dst, int nx, int ny, int nz,
                                                     size_t N, int chunks_per_row, unsigned total_waves, unsigned tune,
                                                     StepCoef<typename ST::comp, VS::Q> k, int closure,
                                                     const float *__restrict__ ghost, FaceTab<VS::Q> ft,
                                                     FieldCoef<VS::Q> fk, int sponge_width, double sponge_sigma) {
    const int lane = threadIdx.x & 63;
    const unsigned wid = (unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool ntl = (tune & kTuneNtLoad) != 0, nts = (tune & kTuneNtStore) != 0;
    const unsigned G = gridDim.x * 4u;
    unsigned wave = blockIdx.x * 4u + wid;
    if (wave >= total_waves) return;
    const OpenEdge<VS::Q, LAYER> edge{closure, ghost, ft, fk, sponge_width, sponge_sigma};
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
                                                        (int)(wave % (unsigned)chunks_per_row), lane, nts, k, cur,
                                                        edge);
        if (!more) break;
        cur = nxt;
        wave = wn;
    }
}

// ------------------------------------------------------------------ sponge layer

// Grid (x blocks, 2D slabs): slab f = 2a + side holds the cells within W of face f that are not
// in a slab of a lower axis, so every layer cell is visited exactly once and the interior not at all.
template <class VS, class ST>
__global__ __launch_bounds__(256) void sponge_kernel(typename ST::elem *__restrict__ g, size_t N, int nx, int ny,
                                                     int nz, int width, double sigma_max) {
    using CT = typename ST::comp;
    const int n[3] = {nx, ny, nz};
    const int f = blockIdx.y, a = f >> 1, side = f & 1;
    const int wa = min(width, n[a]);  // slab depth
    int ext[3], lo[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (b == a) {
            ext[b] = wa;
            lo[b] = side ? n[b] - wa : 0;
        } else if (b < a && b < VS::D) {  // the slabs of axis b own its first and last W cells
            const int wb = min(width, n[b]);
            ext[b] = max(n[b] - 2 * wb, 0);
            lo[b] = wb;
        } else {
            ext[b] = n[b];
            lo[b] = 0;
        }
    }
    if (side == 1 && 2 * wa > n[a]) {  // thin box: the low slab already covers the overlap
        ext[a] = n[a] - wa;
        lo[a] = wa;
    }
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)ext[0] * ext[1] * ext[2]) return;
    const long long r = t / ext[0];
    const int x = (int)(t - r * ext[0]) + lo[0];
    const int y = (int)(r % ext[1]) + lo[1];
    const int z = (int)(r / ext[1]) + lo[2];
    int d = min(x, nx - 1 - x);
    if (VS::D >= 2) d = min(d, min(y, ny - 1 - y));
    if (VS::D >= 3) d = min(d, min(z, nz - 1 - z));
    if (d >= width) return;
    const size_t cell = ((size_t)z * ny + y) * nx + x;
    const CT fac = sponge_factor<CT>(d, width, sigma_max);
#pragma unroll
    for (int i = 0; i < VS::Q; ++i) {
        typename ST::elem *p = g + (size_t)i * N + cell;
        *p = sponge_damp<ST>(*p, fac);
    }
}

// ------------------------------------------------------------------ network ghosts
// Every face node: [strip(t), strip(t-1)] (each 3 cells x Q populations, canonical order, physical
// units) -> network -> the K entering populations (physical units) into ghost[node * K + r], limited in
// energy: with E_in = sum_r y_r^2 / f*, E_out = sum over the node's populations leaving through
// the face (canonical c_x = -1) of g^2 / f*, and n the number of faces the node lies on, y is
// scaled by sqrt(B / E_in) when E_in > B = E_out / (2^n - 1).  Each ghost value pulled into the
// box belongs to one node, and a face prediction feeds at most (2^n - 1) / n of its energy into
// the box (means over faces), so the energy entering at a node never exceeds the energy leaving
// it: the open box cannot gain energy at tau = 1/2 whatever the network predicts.
template <class VS, class ST, bool HIST>
__global__ __launch_bounds__(256) void ghost_mlp_kernel(const typename ST::elem *__restrict__ src, size_t N,
                                                        const float *__restrict__ P, float *__restrict__ ghost,
                                                        const float *__restrict__ hist_in, float *__restrict__ hist_out,
                                                        FaceTab<VS::Q> ft, FieldCoef<VS::Q> fk) {
    static_assert(NetGeom<VS>::fits, "network tiles");
    using G = NetGeom<VS>;
    constexpr int NS = G::NSTRIP;
    __shared__ FwdTiles<G::ZW> tiles[4];
    __shared__ float pred[4][16][G::NOUT];
    __shared__ NetFrags<VS> F;
    // per face f and canonical population j: the face population, its decode factor and 1/f*
    __shared__ int perm_s[6][VS::Q];
    __shared__ float dec_s[6][VS::Q], invf_s[6][VS::Q];
    for (int t = threadIdx.x; t < 6 * VS::Q; t += 256) {
        const int f = t / VS::Q, j = t - f * VS::Q;
        const int i = f < ft.nfaces ? ft.perm[f][j] : 0;
        perm_s[f][j] = i;
        dec_s[f][j] = (float)fk.dec[i];
        invf_s[f][j] = (float)(1.0 / fk.f[i]);
    }
    stage_forward_weights<VS>(P, F);  // ends with a block barrier
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    FwdView<G::ZW> T = fwd_view(tiles[wid]);
    const long long count = ft.node_off[ft.nfaces];
    const long long ntiles = (count + 15) / 16;
    for (long long tile = (long long)blockIdx.x * 4 + wid; tile < ntiles; tile += (long long)gridDim.x * 4) {
        const long long base = tile * 16;
        const int nrows = (int)min((long long)16, count - base);
        // the node of this lane's row
        int p[3];
        const int r = lane & 15, g = lane >> 4;
        const bool row_ok = r < nrows;
        const long long node = base + (row_ok ? r : 0);
        const int f = node_cell(ft, node, p);
        const int a = f >> 1, step = (f & 1) ? -1 : 1;
        const size_t cell0 = ((size_t)p[2] * ft.n[1] + p[1]) * ft.n[0] + p[0];
        const long long stride_a = a == 0 ? 1 : (a == 1 ? (long long)ft.n[0] : (long long)ft.n[0] * ft.n[1]);
        auto strip_now = [&](int v) {  // value v of this node's current strip
            const int m = v / VS::Q, j = v - m * VS::Q;
            const size_t cell = (size_t)((long long)cell0 + (long long)(m * step) * stride_a);
            return dec_s[f][j] * (float)ST::dec(src[(size_t)perm_s[f][j] * N + cell]);
        };
        // input [strip(t), strip(t-1)]; the previous strip comes from the history buffer (HIST),
        // else the current one stands in; this step's strip becomes the next step's history (the
        // other buffer of the pair).  History layout: value v of node n at v * count + n, so the
        // 16 consecutive nodes of a tile read and write 64 contiguous bytes per value.  Every lane
        // of a load loads (padding values and rows past the tile's read a valid value, then scaled
        // by 0; kept values are scaled by 1, exactly), so no load sits in a lane-dependent branch
        // and none waits for another; with the history, the loads of columns 4t .. 4t + 3 skip the
        // strip when all four are history columns, and the history when none is.
        float now[tile_vals<VS>()], before[tile_vals<VS>()], vals[tile_vals<VS>()];
#pragma unroll
        for (int t = 0; t < tile_vals<VS>(); ++t) {
            const int v = g + 4 * t, vv = v < G::NIN ? v : G::NIN - 1;
            if (!HIST || 4 * t < NS) now[t] = strip_now(vv < NS ? vv : vv - NS);
            if constexpr (HIST) {
                if (4 * t + 3 >= NS) before[t] = hist_in[(long long)(vv < NS ? 0 : vv - NS) * count + node];
            }
        }
#pragma unroll
        for (int t = 0; t < tile_vals<VS>(); ++t) {
            const int v = g + 4 * t, vv = v < G::NIN ? v : G::NIN - 1;
            const float x = HIST && vv >= NS ? before[t] : now[t];
            vals[t] = x * ((row_ok && v < G::NIN) ? 1.0f : 0.0f);
            if (row_ok && v < NS) hist_out[(long long)v * count + node] = vals[t];
        }
        float mx = 0.0f, e_out = 0.0f;
        const float s = normalise_tile<VS>(
            T, lane, vals, [&](int v) { return v < VS::Q && VS::cx(v) == -1 ? invf_s[f][v] : 0.0f; }, &mx, &e_out);
        const floatx4 y = net_forward_tile_staged<VS>(F, T, lane);
        const int col = lane & 15;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = 4 * (lane >> 4) + e;
            const float srow = __shfl(s, row, 64);
            if (row < nrows && col < G::NOUT) pred[wid][row][col] = srow * y[e];
        }
        wave_lds_sync();
        if (lane < nrows) {  // lane == r: this lane's node is row `lane`; energies in units of mx^2
            float e_in = 0.0f;
#pragma unroll
            for (int k = 0; k < G::NOUT; ++k) {
                const float v = pred[wid][lane][k] / mx;
                e_in += v * v * invf_s[f][entering_index<VS>(k)];
            }
            int nf = 0;
            for (int b = 0; b < VS::D; ++b) nf += (p[b] == 0) + (p[b] == ft.n[b] - 1);
            const float budget = e_out / (float)((1 << nf) - 1);
            const float sc = e_in > budget ? sqrtf(budget / e_in) : 1.0f;
#pragma unroll
            for (int k = 0; k < G::NOUT; ++k) ghost[(base + lane) * G::NOUT + k] = sc * pred[wid][lane][k];
        }
        wave_lds_sync();
    }
}

// ------------------------------------------------------------------ 2D open box, one launch per step
// The step of a 2D open box as a single launch: blocks [0, face_blocks) recompute the ring (the
// cells on a face), the blocks after them step the interior cells 0 < x < nx - 1, 0 < y < ny - 1
// as the generic step kernel does.  Ring cells are owned as by the shell kernel: the x faces
// hold their corners, the y faces the cells 0 < x < nx - 1 between them.
//
// With MLP every wave owns a segment of at most kOpenSeg ring cells of one face.  It evaluates
// the network for the face nodes those cells pull from (rows of one 16-row tile): the segment's
// own nodes and one more on each side, and, for a segment holding a corner cell of an x face,
// the two nodes of the y face nearest that corner.  Predictions stay in LDS; each lane then
// recomputes one ring cell.  Each network row depends on its own node only, so the values,
// the ghost buffer and the history strips equal those of the separate network kernel (rows of
// nodes that two waves evaluate are written twice with equal values).
constexpr int kOpenSeg = 10;
constexpr int kOpenCells = 2;  // interior cells per thread and pass
static_assert(kOpenSeg + 2 + 4 <= 16, "a segment's rows must fit one 16-row tile");

struct OpenSeg {
    int f, p0, m;  // face, first owned in-face position, owned cells
};
struct OpenRows {
    int f, lo, nsame, cA, cB, nrows;  // see open2d_rows
};

// Owned in-face positions of face f: y in [0, ny) on the x faces, x in [1, nx - 1) on the y faces.
__host__ __device__ inline void open2d_owned(int f, int nx, int ny, int &p_lo, int &p_end) {
    p_lo = f < 2 ? 0 : 1;
    p_end = f < 2 ? ny : nx - 1;
}
__host__ __device__ inline int open2d_face_segments(int f, int nx, int ny) {
    int lo, end;
    open2d_owned(f, nx, ny, lo, end);
    return (end - lo + kOpenSeg - 1) / kOpenSeg;
}
__host__ __device__ inline int open2d_segments(int nx, int ny) {
    int n = 0;
    for (int f = 0; f < 4; ++f) n += open2d_face_segments(f, nx, ny);
    return n;
}
__host__ __device__ inline OpenSeg open2d_segment(int w, int nx, int ny) {
    OpenSeg sg{0, 0, 0};
    for (int f = 0; f < 4; ++f) {
        const int nf = open2d_face_segments(f, nx, ny);
        if (w < nf) {
            int lo, end;
            open2d_owned(f, nx, ny, lo, end);
            sg.f = f;
            sg.p0 = lo + w * kOpenSeg;
            sg.m = min(kOpenSeg, end - sg.p0);
            return sg;
        }
        w -= nf;
    }
    return sg;
}
// Rows [0, nsame): nodes lo + j of the segment's face; rows cA, cA + 1 (cA >= 0 when the
// segment holds the corner at y = 0 of an x face): y-low nodes at the corner's x and one
// inward; rows cB, cB + 1 likewise for the corner at y = ny - 1 (y-high nodes).
__host__ __device__ inline OpenRows open2d_rows(const OpenSeg &sg, int nx, int ny) {
    OpenRows r;
    r.f = sg.f;
    const int nface = sg.f < 2 ? ny : nx;
    r.lo = max(sg.p0 - 1, 0);
    r.nsame = min(sg.p0 + sg.m, nface - 1) - r.lo + 1;
    int n = r.nsame;
    r.cA = r.cB = -1;
    if (sg.f < 2 && sg.p0 == 0) {
        r.cA = n;
        n += 2;
    }
    if (sg.f < 2 && sg.p0 + sg.m == ny) {
        r.cB = n;
        n += 2;
    }
    r.nrows = n;
    return r;
}
__host__ __device__ inline void open2d_row_node(const OpenRows &r, int j, int nx, int &f, int &p) {
    if (j < r.nsame) {
        f = r.f;
        p = r.lo + j;
        return;
    }
    const int x0 = r.f == 0 ? 0 : nx - 1, dir = r.f == 0 ? 1 : -1;
    if (r.cA >= 0 && j < r.cA + 2) {
        f = 2;
        p = x0 + dir * (j - r.cA);
    } else {
        f = 3;
        p = x0 + dir * (j - r.cB);
    }
}
// Row of face fb's node at clamp position cl, for a source of a cell of the segment.
__host__ __device__ inline int open2d_row_of(const OpenRows &r, int fb, const int (&cl)[3], int nx) {
    if (fb == r.f) return (fb < 2 ? cl[1] : cl[0]) - r.lo;
    const int d = r.f == 0 ? cl[0] : nx - 1 - cl[0];
    return (fb == 2 ? r.cA : r.cB) + d;
}
// Ring cell c (0 <= c < 2 ny + 2 (nx - 2)) in the ownership order.
__host__ __device__ inline void open2d_ring_cell(long long c, int nx, int ny, int (&x)[3]) {
    x[2] = 0;
    if (c < ny) {
        x[0] = 0;
        x[1] = (int)c;
    } else if (c < 2LL * ny) {
        x[0] = nx - 1;
        x[1] = (int)(c - ny);
    } else if (c < 2LL * ny + (nx - 2)) {
        x[0] = 1 + (int)(c - 2LL * ny);
        x[1] = 0;
    } else {
        x[0] = 1 + (int)(c - 2LL * ny - (nx - 2));
        x[1] = ny - 1;
    }
}

// Two 16 x 64 tiles per wave (rows padded as FwdTiles'): the network's input z and its second
// hidden layer h2 share one (z is dead once the first layer has read it).
struct Open2dTiles {
    unsigned short (&z)[16][64 + kTilePad];
    unsigned short (&h1)[16][64 + kTilePad];
    unsigned short (&h2)[16][64 + kTilePad];
};

// LDS of a block of the ring with MLP.
template <class VS>
struct Open2dShared {
    NetFrags<VS> F;
    alignas(16) unsigned short zt[4][16][64 + kTilePad];  // 16-byte aligned rows: the network's 16-byte operand reads
    alignas(16) unsigned short h1t[4][16][64 + kTilePad];
    float pred[4][16][NetGeom<VS>::NOUT];
    float predp[4][16][VS::Q];  // limited predictions by population: the row's value for rank[face][i]
    int perm[4][VS::Q], rank[4][VS::Q];
    float dec[VS::Q], invf[VS::Q];  // by population
};

// HIST: the previous strips come from hist_in (else the current strips stand in for them).
template <class VS, class ST, bool SKIP0, bool HALF, bool HIST>
__device__ void open2d_ring_mlp(Open2dShared<VS> &sh, const typename ST::elem *__restrict__ src,
                                typename ST::elem *__restrict__ dst, size_t N, const float *__restrict__ P,
                                float *__restrict__ ghost, const float *__restrict__ hist_in,
                                float *__restrict__ hist_out, const FaceTab<VS::Q> &ft,
                                const StepCoef<typename ST::comp, VS::Q> &ks, const FieldCoef<VS::Q> &fk,
                                int sponge_width, double sponge_sigma) {
    static_assert(NetGeom<VS>::fits, "network tiles");
    using G = NetGeom<VS>;
    using CT = typename ST::comp;
    static_assert(VS::D == 2 && G::ZW == 64, "2D sets only");
    constexpr int NS = G::NSTRIP, K = G::NOUT;
    NetFrags<VS> &F = sh.F;
    auto &pred = sh.pred;
    auto &perm_s = sh.perm;
    auto &rank_s = sh.rank;
    auto &dec_s = sh.dec;
    auto &invf_s = sh.invf;
    for (int t = threadIdx.x; t < 4 * VS::Q; t += 256) {  // no load here waits for another
        const int f = t / VS::Q, j = t - f * VS::Q;
        perm_s[f][j] = ft.perm[f][j];
        const int rk = ft.rank[f][j];  // rank of population j entering through face f
        rank_s[f][j] = rk < 0 ? 0 : rk;
        if (f == 0) {
            dec_s[j] = (float)fk.dec[j];
            invf_s[j] = (float)(1.0 / fk.f[j]);
        }
    }
    __syncthreads();  // tables visible before the loads below
    const int nx = ft.n[0], ny = ft.n[1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int w = blockIdx.x * 4 + wid;
    const bool active = w < open2d_segments(nx, ny);
    const OpenSeg sg = open2d_segment(active ? w : 0, nx, ny);
    const OpenRows plan = open2d_rows(sg, nx, ny);
    // the loads of this lane's ring cell, of its tile values and of the weights are all issued
    // before the wave waits for any of them
    const bool owner = active && lane < sg.m;
    int xc[3] = {0, 0, 0};
    {
        const int a = sg.f >> 1, q = sg.p0 + (owner ? lane : 0);
        xc[a] = (sg.f & 1) ? (a == 0 ? nx : ny) - 1 : 0;
        xc[1 - a] = q;
    }
    CT s[VS::Q];
    if (owner) shell_inside<VS, ST, SKIP0>(src, N, kBcMlp, xc, ft, s);
    // the tile rows of the face nodes each source of the ring cell lies beyond (-1: not beyond
    // that face), x face first as in shell_outside; computed before the network
    int row_x[VS::Q], row_y[VS::Q];
#pragma unroll
    for (int i = 0; i < VS::Q; ++i) {
        const int sp[2] = {xc[0] - VS::cx(i), xc[1] - VS::cy(i)};
        const int cl[3] = {min(max(sp[0], 0), nx - 1), min(max(sp[1], 0), ny - 1), 0};
        row_x[i] = sp[0] != cl[0] ? open2d_row_of(plan, sp[0] > cl[0] ? 1 : 0, cl, nx) : -1;
        row_y[i] = sp[1] != cl[1] ? open2d_row_of(plan, sp[1] > cl[1] ? 3 : 2, cl, nx) : -1;
    }

    const int r = lane & 15, g = lane >> 4;
    const bool row_ok = active && r < plan.nrows;
    int f, pos;
    open2d_row_node(plan, row_ok ? r : 0, nx, f, pos);
    int p[3] = {0, 0, 0};
    const int a = f >> 1, step = (f & 1) ? -1 : 1;
    p[a] = (f & 1) ? (a == 0 ? nx : ny) - 1 : 0;
    p[1 - a] = pos;
    // node ids run face after face: ny nodes on each x face, nx on each y face
    const long long node = (f < 2 ? (long long)f * ny : 2LL * ny + (long long)(f - 2) * nx) + pos;
    const size_t cell0 = (size_t)p[1] * nx + p[0];
    const long long stride_a = a == 0 ? 1 : (long long)nx;
    auto strip_now = [&](int v) {  // value v of this row's current strip
        const int m = v / VS::Q, j = v - m * VS::Q;
        const size_t cell = (size_t)((long long)cell0 + (long long)(m * step) * stride_a);
        const int i = perm_s[f][j];
        return dec_s[i] * (float)ST::dec(src[(size_t)i * N + cell]);
    };
    // input [strip(t), strip(t-1)]: the previous strip from the history (the current one again on
    // the first step after the state was set); this step's strip becomes the next step's history.
    // Every lane loads (padding values and rows past the tile's read a valid value, later scaled
    // by 0; kept values are scaled by 1, exactly), so no load sits in a branch, and all of them,
    // the ring cell's and the weights' are issued before the first wait.
    // (with the history, as in the network kernel: no strip loads for the columns 4t .. 4t + 3 that
    // are all history columns, no history loads where none is)
    float now[tile_vals<VS>()], before[tile_vals<VS>()];
#pragma unroll
    for (int t = 0; t < tile_vals<VS>(); ++t) {
        const int v = g + 4 * t, vv = v < G::NIN ? v : G::NIN - 1;
        if (!HIST || 4 * t < NS) now[t] = strip_now(vv < NS ? vv : vv - NS);
    }
    const long long count = ft.node_off[ft.nfaces];  // history: value v of node n at v * count + n
    if constexpr (HIST) {
#pragma unroll
        for (int t = 0; t < tile_vals<VS>(); ++t) {
            const int v = g + 4 * t, vv = v < G::NIN ? v : G::NIN - 1;
            if (4 * t + 3 >= NS) before[t] = hist_in[(long long)(vv < NS ? 0 : vv - NS) * count + node];
        }
    } else {
#pragma unroll
        for (int t = 0; t < tile_vals<VS>(); ++t) before[t] = now[t];
    }
    CT enc[VS::Q];  // physical to stored units, for the predictions pulled into the ring cell
#pragma unroll
    for (int i = 0; i < VS::Q; ++i) enc[i] = (CT)fk.enc[i];
    stage_forward_weights<VS>(P, F);  // ends with a block barrier
    if (!active) return;

    float vals[tile_vals<VS>()];
#pragma unroll
    for (int t = 0; t < tile_vals<VS>(); ++t) {
        const int v = g + 4 * t;
        const int vv = v < G::NIN ? v : G::NIN - 1;
        vals[t] = (vv < NS ? now[t] : before[t]) * ((row_ok && v < G::NIN) ? 1.0f : 0.0f);
        if (row_ok && v < NS) hist_out[(long long)v * count + node] = vals[t];
    }
    Open2dTiles T{sh.zt[wid], sh.h1t[wid], sh.zt[wid]};
    float mx = 0.0f, e_out = 0.0f;
    const float sn = normalise_tile<VS>(
        T, lane, vals, [&](int v) { return v < VS::Q && VS::cx(v) == -1 ? invf_s[perm_s[f][v]] : 0.0f; }, &mx,
        &e_out);
    const floatx4 y = net_forward_tile_staged<VS>(F, T, lane);
    const int col = lane & 15;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = 4 * (lane >> 4) + e;
        const float srow = __shfl(sn, row, 64);
        if (row < plan.nrows && col < K) pred[wid][row][col] = srow * y[e];
    }
    wave_lds_sync();
    if (lane < plan.nrows) {  // lane == r: energies of this row's node in units of mx^2
        float e_in = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float v = pred[wid][lane][k] / mx;
            e_in += v * v * invf_s[perm_s[f][entering_index<VS>(k)]];
        }
        const int nf = (p[0] == 0) + (p[0] == nx - 1) + (p[1] == 0) + (p[1] == ny - 1);
        const float budget = e_out / (float)((1 << nf) - 1);
        const float sc = e_in > budget ? sqrtf(budget / e_in) : 1.0f;
        float gv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            gv[k] = sc * pred[wid][lane][k];
            ghost[node * K + k] = gv[k];
        }
#pragma unroll
        for (int i = 0; i < VS::Q; ++i) {
            const int rk = rank_s[f][i];
            float v = gv[0];
#pragma unroll
            for (int k = 1; k < K; ++k) v = rk == k ? gv[k] : v;
            sh.predp[wid][lane][i] = v;
        }
    }
    wave_lds_sync();
    if (!owner) return;
    // the closure's values, as shell_outside forms them (mean over the faces, then to stored units;
    // division by a count of 1 or 2 is exact as the identity or a product with 1/2)
#pragma unroll
    for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
        if (row_x[i] < 0 && row_y[i] < 0) continue;
        float acc = 0.0f;
        int cnt = 0;
        if (row_x[i] >= 0) {
            acc += sh.predp[wid][row_x[i]][i];
            ++cnt;
        }
        if (row_y[i] >= 0) {
            acc += sh.predp[wid][row_y[i]][i];
            ++cnt;
        }
        s[i] = (CT)(cnt == 2 ? acc * 0.5f : acc) * enc[i];
    }
    collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(ks, s);
    const size_t cell = (size_t)xc[1] * nx + xc[0];
    if (sponge_width > 0) {  // a sponge layer behind the network: ring cells lie at distance 0
        const CT fac = sponge_factor<CT>(0, sponge_width, sponge_sigma);
#pragma unroll
        for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) dst[(size_t)i * N + cell] = sponge_damp<ST>(ST::enc(s[i]), fac);
    } else {
#pragma unroll
        for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) dst[(size_t)i * N + cell] = ST::enc(s[i]);
    }
}

template <class VS, class ST, bool SKIP0, bool HALF, bool MLP>
__global__ __launch_bounds__(256) void open_step_2d(const typename ST::elem *__restrict__ src,
                                                    typename ST::elem *__restrict__ dst, size_t N, int closure,
                                                    int face_blocks, const float *__restrict__ P,
                                                    float *__restrict__ ghost, const float *__restrict__ hist_in,
                                                    float *__restrict__ hist_out, FaceTab<VS::Q> ft,
                                                    StepCoef<typename ST::comp, VS::Q> k,
                                                    StepCoef<typename ST::comp, VS::Q> ks, FieldCoef<VS::Q> fk,
                                                    int sponge_width, double sponge_sigma) {
    using CT = typename ST::comp;
    static_assert(VS::D == 2, "2D sets only");
    const int nx = ft.n[0], ny = ft.n[1];
    // A sponge layer (sponge_width > 0: the sponge closure, or a layer behind the network): each
    // cell within sponge_width of a face is damped as the sponge kernel damps it, right after its
    // new state is stored (same values: decode, scale, encode)
    auto store = [&](size_t cell, int x, int y, const CT (&s)[VS::Q], auto encode) {
        const int d = min(min(x, nx - 1 - x), min(y, ny - 1 - y));
        if (d < sponge_width) {
            const CT fac = sponge_factor<CT>(d, sponge_width, sponge_sigma);
#pragma unroll
            for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) dst[(size_t)i * N + cell] = sponge_damp<ST>(encode(s[i]), fac);
        } else {
#pragma unroll
            for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) dst[(size_t)i * N + cell] = encode(s[i]);
        }
    };
    if ((int)blockIdx.x < face_blocks) {
        if constexpr (MLP) {
            __shared__ Open2dShared<VS> sh;
            if (hist_in)
                open2d_ring_mlp<VS, ST, SKIP0, HALF, true>(sh, src, dst, N, P, ghost, hist_in, hist_out, ft, ks, fk,
                                                           sponge_width, sponge_sigma);
            else
                open2d_ring_mlp<VS, ST, SKIP0, HALF, false>(sh, src, dst, N, P, ghost, hist_in, hist_out, ft, ks, fk,
                                                            sponge_width, sponge_sigma);
        } else {
            const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
            if (c >= 2LL * ny + 2LL * (nx - 2)) return;
            int x[3];
            open2d_ring_cell(c, nx, ny, x);
            CT s[VS::Q];
            shell_inside<VS, ST, SKIP0>(src, N, closure, x, ft, s);
            collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(ks, s);
            store((size_t)x[1] * nx + x[0], x[0], x[1], s, [](CT v) { return ST::enc(v); });
        }
        return;
    }
    // interior cells, kOpenCells per thread and pass (the loads of all of them in flight together;
    // a cell past the end loads a valid cell and stores nothing), grid-stride over the blocks
    // after the ring's
    const size_t mx = (size_t)(nx - 2), interior = mx * (size_t)(ny - 2);
    const size_t stride = (size_t)(gridDim.x - face_blocks) * 256u;
    for (size_t t0 = (size_t)(blockIdx.x - face_blocks) * 256u + threadIdx.x; t0 < interior;
         t0 += kOpenCells * stride) {
        CT s[kOpenCells][VS::Q];
        size_t cell[kOpenCells];
        int cx[kOpenCells], cy[kOpenCells];
#pragma unroll
        for (int c = 0; c < kOpenCells; ++c) {
            const size_t t = t0 + c * stride < interior ? t0 + c * stride : t0;
            int x, y;
            if (interior <= 0xffffffffull) {  // 32-bit division when it fits
                x = 1 + (int)((unsigned)t % (unsigned)mx);
                y = 1 + (int)((unsigned)t / (unsigned)mx);
            } else {
                x = 1 + (int)(t % mx);
                y = 1 + (int)(t / mx);
            }
            cell[c] = (size_t)y * nx + x;
            cx[c] = x;
            cy[c] = y;
            s[c][0] = 0;
#pragma unroll
            for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i)
                s[c][i] = dec_io<ST, ST::has_raw>(src[(size_t)i * N + (size_t)(y - VS::cy(i)) * nx + (x - VS::cx(i))]);
        }
#pragma unroll
        for (int c = 0; c < kOpenCells; ++c) {
            collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(k, s[c]);
            if (t0 + c * stride < interior) {
                store(cell[c], cx[c], cy[c], s[c], [](CT v) { return enc_io<ST, ST::has_raw>(v); });
            }
        }
    }
}

// ------------------------------------------------------------------ training pairs
// For inner-box face nodes (ids in the inner box's numbering), read the state of a larger
// run whose cell origin + x is inner cell x: the strip at the node (one time level, NSTRIP
// values at strips + t * stride) and the entering populations at the node's outside neighbour
// (targets, skipped when NULL), physical units.  Ids outside the face-node range give zeros.
template <class VS, class ST>
__global__ __launch_bounds__(256) void gather_pairs_kernel(const typename ST::elem *__restrict__ src, size_t N,
                                                           int onx, int ony, int ox, int oy, int oz,
                                                           const long long *__restrict__ ids, long long count,
                                                           float *__restrict__ strips, long long stride,
                                                           float *__restrict__ targets, FaceTab<VS::Q> ft,
                                                           FieldCoef<VS::Q> fk) {
    using G = NetGeom<VS>;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= count) return;
    float *row = strips + t * stride;
    const long long id = ids[t];
    if (id < 0 || id >= ft.node_off[ft.nfaces]) {  // not a face node: zeros
        for (int v = 0; v < G::NSTRIP; ++v) row[v] = 0.0f;
        if (targets)
            for (int r = 0; r < G::NOUT; ++r) targets[t * G::NOUT + r] = 0.0f;
        return;
    }
    int p[3];
    const int f = node_cell(ft, id, p);
    const int a = f >> 1, step = (f & 1) ? -1 : 1;
    const int o[3] = {ox, oy, oz};
    auto outer_cell = [&](const int (&q)[3]) {
        return ((size_t)(q[2] + o[2]) * ony + (q[1] + o[1])) * onx + (q[0] + o[0]);
    };
    for (int m = 0; m < 3; ++m) {
        int q[3] = {p[0], p[1], p[2]};
        q[a] += m * step;
        const size_t cell = outer_cell(q);
        for (int j = 0; j < VS::Q; ++j) {
            const int i = ft.perm[f][j];
            row[m * VS::Q + j] = (float)fk.dec[i] * (float)ST::dec(src[(size_t)i * N + cell]);
        }
    }
    if (!targets) return;
    int q[3] = {p[0], p[1], p[2]};
    q[a] -= step;  // the outside neighbour
    const size_t gcell = outer_cell(q);
    for (int r = 0; r < G::NOUT; ++r) {
        const int i = ft.perm[f][entering_index<VS>(r)];
        targets[t * G::NOUT + r] = (float)(fk.dec[i] * (double)ST::dec(src[(size_t)i * N + gcell]));
    }
}

// ------------------------------------------------------------------ field comparison
// Partials of { sum (a - b)^2, sum b^2, max |a - b| } of a box field a against field b of a
// larger box at offset origin.
[[maybe_unused]] static __global__ __launch_bounds__(256) void compare_partials(const double *__restrict__ A, int nx, int ny, int nz,
                                                        const double *__restrict__ B, int bnx, int bny, int ox, int oy,
                                                        int oz, double *__restrict__ part) {
    double v[3] = {0, 0, 0};
    const bool is_max[3] = {false, false, true};
    const size_t N = (size_t)nx * ny * nz;
    for (size_t cell = (size_t)blockIdx.x * 256 + threadIdx.x; cell < N; cell += (size_t)gridDim.x * 256) {
        const int x = (int)(cell % nx);
        const size_t r = cell / nx;
        const int y = (int)(r % ny), z = (int)(r / ny);
        const double b = B[((size_t)(z + oz) * bny + (y + oy)) * bnx + (x + ox)];
        const double d = A[cell] - b;
        v[0] += d * d;
        v[1] += b * b;
        v[2] = fmax(v[2], fabs(d));
    }
    block_reduce<3>(v, is_max);
    if (threadIdx.x == 0)
        for (int j = 0; j < 3; ++j) part[3 * blockIdx.x + j] = v[j];
}

}  // namespace lbm
