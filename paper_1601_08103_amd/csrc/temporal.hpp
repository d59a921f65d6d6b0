// Two time steps per launch (temporal blocking) for periodic boxes.
//
// The pull update of Section "The lattice Boltzmann scheme" reads, for every cell, population
// i of the neighbour x - c_i; two updates in a row therefore need the state of step t on the
// cells within two stencil hops of a tile, and the state of step t+1 within one hop.  One
// block owns a tile of the box and marches along the last axis ("march" axis z in 3D, y in
// 2D), one plane at a time:
//   phase A (plane p):   step t -> t+1 on the tile plus a one-cell ring (read from HBM),
//   phase B (plane p-1): step t+1 -> t+2 on the tile (read from phase A's results),
// so the state goes through HBM once per two steps: read once (plus the ring and two warm-up
// planes per segment) and written once.  Populations that move within the plane are exchanged
// between threads through LDS rings of 3 + c_z planes; populations with c_x = c_y = 0 stay in
// the registers of the thread that owns the column.  The loads of the next two planes (one for
// the sets with 13 and more velocities) are in flight while a plane is computed, and one
// barrier per plane orders the LDS traffic.  Each step's results are rounded to the
// storage type exactly as a store and reload would (encode, decode), and every cell goes
// through the same collision as the one-step kernels, so two steps here give the same bits as
// two one-step launches.
#pragma once

#include "kernels.hpp"

namespace lbm {

// Velocities in the kernel frame: 3D (cx, cy, cz); 2D (cx, 0, cy), marching along y.
template <class VS>
struct TbFrame {
    static_assert(VS::D >= 2, "temporal blocking marches along the last of two or three axes");
    static constexpr int kx(int i) { return VS::cx(i); }
    static constexpr int ky(int i) { return VS::D == 3 ? VS::cy(i) : 0; }
    static constexpr int kz(int i) { return VS::D == 3 ? VS::cz(i) : VS::cy(i); }
    static constexpr bool moves_xy(int i) { return kx(i) != 0 || ky(i) != 0; }
    // a population with march-axis component c_z is read c_z planes behind, by phase B one
    // plane behind phase A: ring of 3 + c_z slots (one more than the planes in use, see below)
    static constexpr int depth(int i) { return 3 + kz(i); }
    static constexpr bool y_halo() {
        for (int i = 0; i < VS::Q; ++i)
            if (ky(i) != 0) return true;
        return false;
    }
    static constexpr int plane_off(int i) {
        int o = 0;
        for (int j = 0; j < i; ++j)
            if (moves_xy(j)) o += depth(j);
        return o;
    }
    static constexpr int planes() { return plane_off(VS::Q); }
    // the population with c_x = c_y = 0 and c_z = dz, or -1
    static constexpr int local(int dz) {
        for (int i = 0; i < VS::Q; ++i)
            if (!moves_xy(i) && kz(i) == dz) return i;
        return -1;
    }
};

// Tile shape per (set, storage): 64 cells along x; in 3D the largest TY in {16, 8, 4} whose
// LDS rings fit kTbLdsBudget, 32 TY threads with two interior columns each; in 2D one row of
// 64 columns per block of 64 threads.  TY = 0: no shape fits (the variant is unsupported).
constexpr int kTbTx = 64;
constexpr int kTbLdsBudget = 64 * 1024;

template <class VS, class ST>
struct TbShape {
    using F = TbFrame<VS>;
    static constexpr int hy = F::y_halo() ? 1 : 0;
    static constexpr long lds_bytes(int ty) {
        return (long)F::planes() * (kTbTx + 2) * (ty + 2 * hy) * (long)sizeof(typename ST::elem);
    }
    static constexpr int pick() {
        if (VS::D == 2) return lds_bytes(1) <= kTbLdsBudget ? 1 : 0;
        for (int ty = 16; ty >= 4; ty /= 2)
            if (lds_bytes(ty) <= kTbLdsBudget) return ty;
        return 0;
    }
    static constexpr int TY = pick();
    // two interior columns per thread in 3D, one in 2D
    static constexpr int NT = VS::D == 2 ? 64 : (TY > 0 ? 32 * TY : 64);
    // waves per SIMD the register budget is set for (4: 128 VGPRs; 2 for the sets with 13 or
    // more velocities, whose two collisions per column need more), lowered where the LDS
    // (160 KB per CU) holds fewer blocks than that needs
    static constexpr int blocks_by_lds() { return TY == 0 ? 1 : (int)(160 * 1024 / lds_bytes(TY)); }
    static constexpr int wpe() {
        const int cap = VS::Q >= 13 ? 2 : 4;
        const int w = blocks_by_lds() * NT / 256;
        return w < 1 ? 1 : w > cap ? cap : w;
    }
    static constexpr int WPE = wpe();
};

// Raw buffer access: a block-uniform descriptor for one plane of one population (base address,
// no stride, 2^32 - 1 bytes, gfx9 word 3) and a 32-bit byte offset per lane, so a load or store
// is one instruction with no per-lane 64-bit address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, -1, 0x00020000);
}

template <typename E>
__device__ __forceinline__ E buf_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (sizeof(E) == 2) {
        return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0));
    } else if constexpr (sizeof(E) == 4) {
        return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    } else {
        return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    }
}

template <typename E>
__device__ __forceinline__ void buf_store(E v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (sizeof(E) == 2) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)off, 0, 0);
    } else if constexpr (sizeof(E) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
    } else {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)off, 0, 0);
    }
}

template <class VS, class ST, bool SKIP0, bool HALF, int TY, int NT, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void step_tb2(const typename ST::elem *__restrict__ src,
                                               typename ST::elem *__restrict__ dst, int fx, int fy, int fz,
                                               size_t N, int sz, int tiles_x, int tiles_y,
                                               StepCoef<typename ST::comp, VS::Q> k) {
    using F = TbFrame<VS>;
    using E = typename ST::elem;
    using CT = typename ST::comp;
    constexpr bool RAW = ST::has_raw;
    constexpr int Q = VS::Q;
    constexpr int i0 = SKIP0 ? 1 : 0;
    constexpr int TX = kTbTx;
    constexpr int HY = F::y_halo() ? 1 : 0;
    constexpr int DX = TX + 2, DY = TY + 2 * HY, PL = DX * DY;
    constexpr int NJ = TX * TY / NT;  // interior columns per thread
    static_assert(NJ * NT == TX * TY && NJ >= 1, "tile and block size");
    constexpr int H = PL - TX * TY;    // columns of the ring around the tile
    constexpr int NH = (H + NT - 1) / NT;
    constexpr int NC = NJ + NH;
    constexpr int IU = F::local(1);                  // c = (0, 0, +1): read two planes later
    constexpr int ID = F::local(-1);                 // c = (0, 0, -1): read in the same iteration
    constexpr int IR = SKIP0 ? -1 : F::local(0);     // the rest population, when it is updated
    static_assert(F::planes() > 0, "some population moves within the plane");
    // planes of loads in flight: two where the registers allow (up to 9 velocities)
    constexpr int PF = Q <= 9 ? 2 : 1;
    __shared__ E ring[F::planes() * PL];

    // tile of this block; consecutive tiles on one XCD (blocks go round-robin over the 8 XCDs)
    unsigned b = blockIdx.x;
    if ((gridDim.x & 7u) == 0) b = (b & 7u) * (gridDim.x >> 3) + (b >> 3);
    const int tx = (int)(b % (unsigned)tiles_x);
    const unsigned rr = b / (unsigned)tiles_x;
    const int ty = (int)(rr % (unsigned)tiles_y);
    const int tz = (int)(rr / (unsigned)tiles_y);
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * sz;
    const int w = min(TX, fx - x0), hgt = min(TY, fy - y0), seg = min(sz, fz - z0);
    const int tid = threadIdx.x;

    // columns of this thread in the dilated tile: NJ interior ones (phase B owns the same), then
    // ring columns; (cxl, cyl) dilated coordinates.  Loads and stores address a plane through a
    // block-uniform base pointer plus a per-column 32-bit offset within the plane (xy offsets
    // of the source cell of each population, and of the column's own cell for the stores).
    int cxl[NC], cyl[NC];
    unsigned xyoff[NC][Q], oxy[NJ];  // byte offsets (the host keeps a plane under 4 GiB)
    bool valid[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        int ax, ay;
        bool ok = true;
        if (c < NJ) {
            const int cc = tid + NT * c;
            ax = cc % TX + 1;
            ay = cc / TX + HY;
        } else {
            const int h = tid + NT * (c - NJ);
            ok = h < H;
            if (HY == 0) {
                ax = h == 0 ? 0 : DX - 1;
                ay = 0;
            } else if (h < DX) {
                ax = h;
                ay = 0;
            } else if (h < 2 * DX) {
                ax = h - DX;
                ay = DY - 1;
            } else {
                const int h2 = h - 2 * DX;
                ax = (h2 & 1) ? DX - 1 : 0;
                ay = 1 + (h2 >> 1);
            }
            if (!ok) ax = ay = 0;
        }
        cxl[c] = ax;
        cyl[c] = ay;
        valid[c] = ok;
        int X = (x0 - 1 + ax) % fx;
        if (X < 0) X += fx;
        int Y = (y0 - HY + ay) % fy;
        if (Y < 0) Y += fy;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            xyoff[c][i] = (unsigned)(wrap_add(Y, -F::ky(i), fy) * fx + wrap_add(X, -F::kx(i), fx)) * (unsigned)sizeof(E);
        if (c < NJ) oxy[c < NJ ? c : 0] = (unsigned)(Y * fx + X) * (unsigned)sizeof(E);
    }
    const size_t plane = (size_t)fx * fy;

    E la[NC][Q], lb[NC][Q];
    auto load_plane = [&](int pl, E(&ld)[NC][Q]) {
        int Z = z0 - 1 + pl;
        if (Z < 0) Z += fz;
        if (Z >= fz) Z -= fz;
#pragma unroll
        for (int i = i0; i < Q; ++i) {
            const auto r = plane_rsrc(src + (size_t)i * N + (size_t)wrap_add(Z, -F::kz(i), fz) * plane);
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (valid[c]) ld[c][i] = buf_load<E>(r, xyoff[c][i]);
        }
    };

    // column-local populations of the interior columns: up ring (planes pl, pl-1, pl-2),
    // rest (pl, pl-1), down (pl)
    CT u0[NJ], u1[NJ], u2[NJ], r0[NJ], r1[NJ], d0[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) u0[j] = u1[j] = u2[j] = r0[j] = r1[j] = d0[j] = 0;

    // LDS ring slot of plane q for a population with march-axis component cz (3 + cz slots)
    auto slot = [](int cz, int q, int q3) { return cz > 0 ? (q & 3) : cz == 0 ? q3 : (q & 1); };

    int m3 = 0;  // pl % 3
    // One iteration: phase A on local plane pl from the loads in cur, then the loads of plane
    // pl + 2 into cur, one barrier, phase B on plane pl - 1.  A wave that leaves phase B early
    // writes plane pl + 1 in the next phase A while others still read planes pl - 2 .. pl: the
    // rings have one slot more than the planes phase B reads, so it never overwrites them.
    auto body = [&](int pl, E(&cur)[NC][Q]) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (!valid[c]) continue;
            CT s[Q];
            s[0] = 0;
#pragma unroll
            for (int i = i0; i < Q; ++i) s[i] = dec_io<ST, RAW>(cur[c][i]);
            collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(k, s);
#pragma unroll
            for (int i = i0; i < Q; ++i) {
                const E e = enc_io<ST, RAW>(s[i]);
                if (F::moves_xy(i)) {
                    ring[(F::plane_off(i) + slot(F::kz(i), pl, m3)) * PL + cyl[c] * DX + cxl[c]] = e;
                } else if (c < NJ) {
                    const int cj = c < NJ ? c : 0;
                    const CT v = dec_io<ST, RAW>(e);
                    if (i == IU) u0[cj] = v;
                    if (i == IR) r0[cj] = v;
                    if (i == ID) d0[cj] = v;
                }
            }
        }
        if (pl + PF <= seg + 1) load_plane(pl + PF, cur);  // PF planes in flight across phase B
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        if (pl >= 2) {
            // phase B: step t+2 on plane z0 - 2 + pl (local plane pl - 1), reading local planes
            // pl - 2 (cz = +1), pl - 1 (cz = 0) and pl (cz = -1)
            const int Zq = z0 - 2 + pl;
            const int m3m1 = m3 == 0 ? 2 : m3 - 1;  // (pl - 1) % 3
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                CT s[Q];
                s[0] = 0;
#pragma unroll
                for (int i = i0; i < Q; ++i) {
                    if (F::moves_xy(i)) {
                        const int q = pl - 1 - F::kz(i);
                        s[i] = dec_io<ST, RAW>(ring[(F::plane_off(i) + slot(F::kz(i), q, m3m1)) * PL +
                                                    (cyl[j] - F::ky(i)) * DX + (cxl[j] - F::kx(i))]);
                    } else {
                        s[i] = i == IU ? u2[j] : i == IR ? r1[j] : d0[j];
                    }
                }
                collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(k, s);
                const int xl = cxl[j] - 1, yl = cyl[j] - HY;
                if (xl < w && yl < hgt) {
#pragma unroll
                    for (int i = i0; i < Q; ++i)
                        buf_store<E>(enc_io<ST, RAW>(s[i]), plane_rsrc(dst + (size_t)i * N + (size_t)Zq * plane), oxy[j]);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            u2[j] = u1[j];
            u1[j] = u0[j];
            r1[j] = r0[j];
        }
        m3 = m3 == 2 ? 0 : m3 + 1;
    };

    load_plane(0, la);
    if constexpr (PF == 2) {
        load_plane(1, lb);  // seg >= 1: planes 0 .. seg + 1 are at least three
        for (int pl = 0; pl <= seg + 1; pl += 2) {
            body(pl, la);
            if (pl + 1 <= seg + 1) body(pl + 1, lb);
        }
    } else {
        for (int pl = 0; pl <= seg + 1; ++pl) body(pl, la);
    }
}

}  // namespace lbm
