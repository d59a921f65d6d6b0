// K time steps per launch (temporal blocking, K = 2 or 3; the ring sets allow 4) for periodic
// boxes.
//
// The pull form of the update of Section "Derivation of the Lattice Boltzmann Equation" reads,
// for every cell, population i of the neighbour x - c_i; K updates in a row therefore need the
// state of step t on the cells within K stencil hops of a tile, the state of step t+1 within
// K-1 hops, and so on.
// One block owns a tile of the box and marches along the last axis ("march" axis z in 3D, y
// in 2D), one plane at a time.  Per iteration, stage s (s = 1..K) computes step t+s on one
// plane of the tile dilated by K-s cells (in x, and in y in 3D), s-1 planes behind stage 1:
//   stage 1 reads the state of step t from HBM,
//   stage s > 1 reads stage s-1's results from LDS and registers,
//   stage K writes step t+K to HBM,
// so the state goes through HBM once per K steps: read once (plus the rings around the tile
// and 2(K-1) warm-up planes per segment) and written once.  Populations that move within the
// plane are exchanged between threads through LDS rings of 2 + c_z planes (3 + c_z for K = 2);
// populations with c_x = c_y = 0 stay in the registers of the thread that owns the column in
// every stage.  The loads of the next two planes (one for the sets with 13 and more velocities)
// are in flight while a plane is computed, and K-1 barriers per iteration order the LDS traffic.
// In 3D each thread's interior cells are an x-adjacent pair read and written with one access of
// two elements per population (so nx must be even; FP32 sets of 13 and more velocities excepted);
// the x-neighbour beyond the pair comes from the neighbouring lane by DPP.
// Every cell goes through the same collision as the one-step kernels.  The intermediate steps
// t+1 .. t+K-1 are never stored, so they stay in the compute type: for FP64 and FP32 storage
// that is the stored value itself and K steps here give the same bits as K one-step launches;
// for the 16-bit formats (FP32 collision) a launch rounds to the storage format once, at step
// t+K, instead of once per step, which divides the number of roundings, the dominant error of
// those formats at tau = 1/2 (nothing damps it), by K.
#pragma once

#include <type_traits>

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
    // a population with march-axis component c_z is read c_z planes behind the plane computed
    // from it: 2 + c_z planes in use; with K = 2 the ring holds one more (see step_tbk)
    static constexpr int depth(int i, int K) { return (K == 2 ? 3 : 2) + kz(i); }
    static constexpr bool y_halo() {
        for (int i = 0; i < VS::Q; ++i)
            if (ky(i) != 0) return true;
        return false;
    }
    static constexpr int plane_off(int i, int K) {
        int o = 0;
        for (int j = 0; j < i; ++j)
            if (moves_xy(j)) o += depth(j, K);
        return o;
    }
    static constexpr int planes(int K) { return plane_off(VS::Q, K); }
    // the population with c_x = c_y = 0 and c_z = dz, or -1
    static constexpr int local(int dz) {
        for (int i = 0; i < VS::Q; ++i)
            if (!moves_xy(i) && kz(i) == dz) return i;
        return -1;
    }
};

// Tile shape per (set, storage, K): TX cells along x and TY along y.  In 3D with three or more
// steps and 4-byte ring elements TX = 128 where the rings fit at TY = 16, else TX = 64; TY is the
// largest in {32 or 16, 8, 4} whose LDS rings (one set per intermediate step) fit the budget (64 KB
// for K = 2, the CU's 160 KB otherwise); TX TY / 2 threads with two interior columns each.  In 2D
// one row of 64 columns per block of 64 threads.  TY = 0: no shape fits (the variant is
// unsupported).
// The loads of a tile's side columns (the rings' cells left and right of the tile) fetch a cache
// line per row for a few bytes; every wave-wide load of a row's interior fetches its row segment
// whole.  The L1-to-L2 request rate per CU is what bounds these kernels (about 80 % of a plain
// copy kernel's rate, measured), so a wider tile, with half the side columns per interior cell,
// runs faster although its rings hold more rows (128 x 16 against 64 x 32).

// Element type of the LDS rings: the storage type where it holds the compute type's values
// exactly (FP64, FP32), the compute type (FP32) for the 16-bit formats, whose intermediate steps
// are not rounded.
template <class ST>
using TbRing = std::conditional_t<ST::scaled, typename ST::comp, typename ST::elem>;

template <class VS, class ST, int K>
struct TbShape {
    using F = TbFrame<VS>;
    static constexpr int hy = F::y_halo() ? 1 : 0;
    static constexpr long budget = K == 2 ? 64 * 1024 : 160 * 1024;
    static constexpr long lds_for(int tx, int ty) {
        long cells = 0;
        for (int s = 1; s < K; ++s) cells += (long)(tx + 2 * (K - s)) * (ty + 2 * hy * (K - s));
        return (long)F::planes(K) * cells * (long)sizeof(TbRing<ST>);
    }
    static constexpr int TX =
        (VS::D == 3 && K >= 3 && sizeof(TbRing<ST>) == 4 && lds_for(128, 16) <= budget) ? 128 : 64;
    static constexpr long lds_bytes(int ty) { return lds_for(TX, ty); }
    static constexpr int pick() {
        if (VS::D == 2) return lds_bytes(1) <= budget ? 1 : 0;
        if (TX == 128) return 16;
        // taller tiles (less ring overhead, one 1024-thread block per CU) pay off for 4- and
        // 8-byte ring elements with three or more steps (measured, D3Q7 256^3)
        const int top = (K >= 3 && sizeof(TbRing<ST>) >= 4) ? 32 : 16;
        for (int ty = top; ty >= 4; ty /= 2)
            if (lds_bytes(ty) <= budget) return ty;
        return 0;
    }
    static constexpr int TY = pick();
    static constexpr int NT = VS::D == 2 ? 64 : (TY > 0 ? TX / 2 * TY : 64);
    // waves per SIMD the register budget is set for (4: 128 VGPRs; 2 for the sets with 13 or
    // more velocities, whose collisions per column need more), lowered where the LDS
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
// no stride, record count = the plane's bytes, gfx9 word 3) and a 32-bit byte offset per lane, so
// a load or store is one instruction with no per-lane 64-bit address arithmetic.  An offset at or
// beyond the record count is out of range: the load returns 0 and the store is dropped, without
// a memory access.  Lanes without a cell to load or store (ring columns past the ring's end,
// cells past a ragged box edge) and prefetches past a segment's last plane use that instead of a
// branch, so every path through the kernel issues the same sequence of memory instructions and
// the compiler's wait counts stay exact (a load skipped on some paths makes it wait for all of
// them at the next use of any).  The host keeps a plane under 2 GiB, below kTbOob.
constexpr unsigned kTbOob = 0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *p, unsigned records) {
    // records is block-uniform; readfirstlane keeps it in a scalar register (a per-lane value
    // would turn every access into a loop over distinct descriptors)
    const int rec = __builtin_amdgcn_readfirstlane((int)records);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, rec, 0x00020000);
}

// Decode a value loaded from HBM for stage 1.  FP32 decodes to itself, so the loaded register
// would stay live through the collision, overlap the next prefetch into the same variable, and
// force a copy (and a wait for that prefetch) at the loop latch; an explicit move into a fresh
// register ends the loaded register's life at the decode.
template <class ST, bool RAW>
__device__ __forceinline__ typename ST::comp dec_loaded(typename ST::elem v) {
    if constexpr (sizeof(typename ST::elem) == 4 && !ST::scaled && !ST::has_raw) {
        float r;
        __asm__("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
        return r;
    } else {
        return dec_io<ST, RAW>(v);
    }
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

// Cache policy of the stores: non-temporal for 2- and 4-byte elements.  The state written at
// step t+K is read again only by the next launch, and stores that allocate in L2 evict the planes
// in flight and the halo cells that neighbouring tiles on the same XCD read shortly after
// (measured at 256^3: 2 % faster for FP32, 8 % for the 16-bit formats; FP64, with half as many
// cells per tile, ran 8 % slower with it).  The loads keep the default policy: the halo rows and
// columns are read by two tiles, and with the non-temporal policy on the loads too the kernel
// runs 1.5 times slower.
template <typename E>
constexpr int kTbStream = sizeof(E) == 8 ? 0 : 2;  // 2: the nt bit of the cache-policy operand

template <typename E>
__device__ __forceinline__ void buf_store(E v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (sizeof(E) == 2) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)off, 0, kTbStream<E>);
    } else if constexpr (sizeof(E) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, kTbStream<E>);
    } else {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)off, 0, kTbStream<E>);
    }
}

// Two consecutive elements at a 2-element-aligned byte offset: one access of 4, 8 or 16 bytes.
template <typename E>
using Vec2 = E __attribute__((ext_vector_type(2)));

template <typename E>
__device__ __forceinline__ Vec2<E> buf_load2(__amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (sizeof(E) == 2) {
        return __builtin_bit_cast(Vec2<E>, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
    } else if constexpr (sizeof(E) == 4) {
        return __builtin_bit_cast(Vec2<E>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    } else {
        return __builtin_bit_cast(Vec2<E>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
    }
}

template <typename E>
__device__ __forceinline__ void buf_store2(Vec2<E> v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    if constexpr (sizeof(E) == 2) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, kTbStream<E>);
    } else if constexpr (sizeof(E) == 4) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)off, 0, kTbStream<E>);
    } else {
        typedef unsigned u4 __attribute__((ext_vector_type(4)));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, (int)off, 0, kTbStream<E>);
    }
}

// Column bookkeeping (frame: the tile dilated by K-1 cells, origin at its corner; the tile's
// own cells start at (K-1, HY (K-1))).  In 3D a thread owns two interior cells: two x-adjacent
// ones (a "pair": TX/2 pairs per row, a wave holds one or two rows), read and written with one
// access of two elements per population, except for FP32 with 13 or more velocities, where the
// pair's registers would spill (the FP32 collision's constants are split in two): there two
// cells TY/2 rows apart, each with its own accesses; in 2D one interior cell.  The rings
// b = 1..K-1 around the tile (b cells out) are spread over NR ring slots per thread, one column
// each (threads past the last ring column have none); stage s works on the interior and the
// rings b <= K - s.
template <int K, int TX_, int TY, int NT, int HY, bool PAIR_>
struct TbCols {
    static constexpr int TX = TX_;
    static constexpr bool PAIR = PAIR_;
    static constexpr int NJ = TX * TY / NT;  // interior cells per thread: 2 in 3D (a pair or two rows), 1 in 2D
    static constexpr int ring_cols(int b) { return HY ? 2 * (TX + 2 * b) + 2 * (TY + 2 * b - 2) : 2; }
    static constexpr int ring_total() {
        int n = 0;
        for (int b = 1; b < K; ++b) n += ring_cols(b);
        return n;
    }
    // Ring slots: with pairs every ring column of every ring shares one pool (ring 1 first), so a
    // thread holds at most ceil(total / NT) of them and a slot's ring is known at run time; else
    // each ring has its own slots (odd rings from the last thread down, even ones from the first
    // up), so a slot's ring is a compile-time constant and the stages it works in cost nothing
    // (fewer registers).
    static constexpr int NH(int b) { return (ring_cols(b) + NT - 1) / NT; }
    static constexpr int NR = [] {
        if (PAIR) return (ring_total() + NT - 1) / NT;
        int n = 0;
        for (int b = 1; b < K; ++b) n += NH(b);
        return n;
    }();
    static constexpr int NC = NJ + NR;
    static constexpr int ring_of(int r) {  // !PAIR: ring of slot r
        int o = 0;
        for (int b = 1; b < K; ++b) {
            if (r < o + NH(b)) return b;
            o += NH(b);
        }
        return K;
    }
    static constexpr int first_of_ring(int b) {
        int o = 0;
        for (int q = 1; q < b; ++q) o += NH(q);
        return o;
    }
};

template <class VS, class ST, bool SKIP0, bool HALF, int K, int TX, int TY, int NT, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void step_tbk(
    const typename ST::elem *__restrict__ src, typename ST::elem *__restrict__ dst, int fx, int fy, int fz, size_t N,
    int sz, int tiles_x, int tiles_y, StepCoef<typename ST::comp, VS::Q> k) {
    using F = TbFrame<VS>;
    using E = typename ST::elem;
    using CT = typename ST::comp;
    using E2 = Vec2<E>;
    constexpr bool RAW = ST::has_raw;
    constexpr int Q = VS::Q;
    constexpr int i0 = SKIP0 ? 1 : 0;
    constexpr int HY = F::y_halo() ? 1 : 0;
    using C = TbCols<K, TX, TY, NT, HY, HY == 1 && (sizeof(E) != 4 || Q <= 9)>;
    constexpr bool PAIR = C::PAIR;
    constexpr int NJ = C::NJ;
    constexpr int NR = C::NR;
    constexpr int NC = C::NC;
    static_assert(NJ * NT == TX * TY && NJ == (HY ? 2 : 1), "tile and block size");
    static_assert(K >= 2 && K <= 4, "two to four steps per launch");
    constexpr int IU = F::local(1);               // c = (0, 0, +1): read two iterations later
    constexpr int ID = F::local(-1);              // c = (0, 0, -1): read in the same iteration
    constexpr int IR = SKIP0 ? -1 : F::local(0);  // the rest population, when it is updated
    static_assert(F::planes(K) > 0, "some population moves within the plane");
    // planes of loads in flight: two where the registers allow (up to 9 velocities)
    constexpr int PF = (Q <= 9 && K <= 3) ? 2 : 1;
    // LDS ring set s (s = 1..K-1) holds stage s's results on the tile dilated by K - s
    auto set_pl = [](int s) { return (TX + 2 * (K - s)) * (TY + 2 * HY * (K - s)); };
    auto set_off = [](int s) {
        int o = 0;
        for (int r = 1; r < s; ++r) o += F::planes(K) * (TX + 2 * (K - r)) * (TY + 2 * HY * (K - r));
        return o;
    };
    constexpr int RING_ELEMS = set_off(K);
    // Index of cell (xs, ys) of ring set s within one plane.  In 3D a row keeps its even x first
    // and its odd x after them, so the two cells of every lane's pair, and their x-neighbours, are
    // consecutive across the lanes (no bank conflicts from the pair's stride of two); in 2D rows
    // are plain.
    auto lidx = [](int s, int xs, int ys) {
        const int dx = TX + 2 * (K - s);  // even
        return PAIR ? ys * dx + (xs & 1) * (dx >> 1) + (xs >> 1) : ys * dx + xs;
    };
    using RE = TbRing<ST>;
    constexpr bool CARRY = !std::is_same_v<RE, E>;  // intermediate steps kept in the compute type
    __shared__ RE ring[RING_ELEMS];

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
    // 3D: the first and the last pair of a row, whose x-neighbour outside the pair is not in
    // the neighbouring lane
    constexpr int PX = TX / 2;  // pairs per row
    const bool row_first = PAIR && tid % PX == 0, row_last = PAIR && tid % PX == PX - 1;

    // Columns: (cxl, cyl) in the frame; rbx = 0 for the interior, the ring for a ring slot, K for
    // a slot without a column.  Loads and stores address a plane through a block-uniform base
    // plus a per-lane 32-bit byte offset within the plane: io[i] the interior's source row at the
    // cell (3D: the pair's first cell; the x-shift of a pair comes from the neighbouring lane),
    // fo[i] the element a first or last pair needs from beyond the neighbouring lane, ro[r][i]
    // the source cell of a ring column, so the store offset of the interior (kTbOob where no
    // access is wanted: out of range, no memory touched).
    int cxl[NC], cyl[NC], rbx[NC];
    // io[j][i]: interior cell j (pairs: one offset for the pair, j = 0)
    constexpr int NIO = PAIR ? 1 : NJ;
    unsigned io[NIO][Q], fo[Q], ro[NR > 0 ? NR : 1][Q], so[NIO];
#pragma unroll
    for (int j = 0; j < NIO; ++j) {
        int ax, ay;
        if constexpr (PAIR) {
            ax = 2 * (tid % PX) + (K - 1);
            ay = tid / PX + (K - 1);
        } else {
            const int cc = tid + NT * j;
            ax = cc % TX + (K - 1);
            ay = HY * (cc / TX + (K - 1));
        }
        for (int c = 0; c < (PAIR ? 2 : 1); ++c) {
            cxl[j + c] = ax + c;
            cyl[j + c] = ay;
            rbx[j + c] = 0;
        }
        int X = (x0 + ax - (K - 1)) % fx;
        if (X < 0) X += fx;
        int Y = (y0 + ay - HY * (K - 1)) % fy;
        if (Y < 0) Y += fy;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int Ys = wrap_add(Y, -F::ky(i), fy);
            // pairs read their own two cells (the x-shift comes from the neighbouring lane)
            io[j][i] = (unsigned)(Ys * fx + wrap_add(X, PAIR ? 0 : -F::kx(i), fx)) * (unsigned)sizeof(E);
            if (PAIR) {
                unsigned f = kTbOob;
                if (F::kx(i) > 0 && row_first) f = (unsigned)(Ys * fx + wrap_add(X, -1, fx)) * (unsigned)sizeof(E);
                if (F::kx(i) < 0 && row_last) f = (unsigned)(Ys * fx + wrap_add(X, 2, fx)) * (unsigned)sizeof(E);
                fo[i] = f;
            }
        }
        // a pair lies wholly inside or wholly outside the box (even fx, even tile origin)
        so[j] = (ax - (K - 1) < w && ay - HY * (K - 1) < hgt) ? (unsigned)(Y * fx + X) * (unsigned)sizeof(E) : kTbOob;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        int h, rb;
        if constexpr (PAIR) {  // one pool, ring 1 first
            h = tid + NT * r;
            rb = 1;
            while (rb < K && h >= C::ring_cols(rb)) {
                h -= C::ring_cols(rb);
                ++rb;
            }
        } else {  // the slot's own ring
            rb = C::ring_of(r);
            h = ((rb & 1) ? NT - 1 - tid : tid) + NT * (r - C::first_of_ring(rb));
            if (h >= C::ring_cols(rb)) rb = K;
        }
        int ax = K - 1, ay = HY * (K - 1);
        if (rb < K) {
            const int W = TX + 2 * rb, lo = K - 1 - rb;
            if (HY == 0) {
                ax = h == 0 ? lo : lo + W - 1;
                ay = 0;
            } else if (h < W) {
                ax = lo + h;
                ay = lo;
            } else if (h < 2 * W) {
                ax = lo + h - W;
                ay = lo + TY + 2 * rb - 1;
            } else {
                const int h2 = h - 2 * W;
                ax = (h2 & 1) ? lo + W - 1 : lo;
                ay = lo + 1 + (h2 >> 1);
            }
        }
        cxl[NJ + r] = ax;
        cyl[NJ + r] = ay;
        rbx[NJ + r] = rb;
        int X = (x0 - (K - 1) + ax) % fx;
        if (X < 0) X += fx;
        int Y = (y0 - HY * (K - 1) + ay) % fy;
        if (Y < 0) Y += fy;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            ro[r][i] = rb < K ? (unsigned)(wrap_add(Y, -F::ky(i), fy) * fx + wrap_add(X, -F::kx(i), fx)) * (unsigned)sizeof(E)
                              : kTbOob;
    }
    const size_t plane = (size_t)fx * fy;
    const unsigned plane_bytes = (unsigned)(plane * sizeof(E));  // <= 2^31 (host check)

    // The loads of one plane: the interior's (a pair, or one element in 2D), the elements beyond
    // the neighbouring lane, the ring columns'.
    struct Loaded {
        E2 pr[PAIR ? Q : 1];     // the pair's two elements
        E in[PAIR ? 1 : NJ][Q];  // single interior cells
        E fx1[PAIR ? Q : 1];     // a first or last pair's element beyond the neighbouring lane
        E rg[NR > 0 ? NR : 1][Q];
    };
    // local plane l is global plane z0 - (K - 1) + l (wrapped).  live = false: a prefetch past
    // the segment's last plane, issued anyway so the load sits outside any branch; its records are
    // empty and it reads nothing.
    Loaded la, lb;
    // Populations [ia, ib) only: a prefetch is spread over the K stages of an iteration (chunk s in
    // stage s), so every stage keeps the memory pipeline busy; issued in one burst, the loads of a
    // whole plane fill the queues, stall the issuing waves and leave the pipeline idle for the
    // rest of the iteration.
    auto load_plane = [&](int l, Loaded &ld, bool live, int ia, int ib) {
        int Z = (z0 - (K - 1) + l) % fz;
        if (Z < 0) Z += fz;
#pragma unroll
        for (int i = i0; i < Q; ++i) {
            if (i < ia || i >= ib) continue;
            const auto r = plane_rsrc(src + (size_t)i * N + (size_t)wrap_add(Z, -F::kz(i), fz) * plane,
                                      live ? plane_bytes : 0u);
            if constexpr (PAIR) {
                ld.pr[i] = buf_load2<E>(r, io[0][i]);
                if (F::kx(i) != 0) ld.fx1[i] = buf_load<E>(r, fo[i]);
            } else {
#pragma unroll
                for (int j = 0; j < NIO; ++j) ld.in[j][i] = buf_load<E>(r, io[j][i]);
            }
#pragma unroll
            for (int q = 0; q < NR; ++q) ld.rg[q][i] = buf_load<E>(r, ro[q][i]);  // 0 where no column
        }
    };

    // column-local results of stage s < K on the thread's columns of stage s + 1: c = (0, 0, +1)
    // for the planes of this and the two previous iterations, the rest for this and the
    // previous one, c = (0, 0, -1) for this one
    CT u0[K][NC], u1[K][NC], u2[K][NC], r0[K][NC], r1[K][NC], d0[K][NC];
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int c = 0; c < NC; ++c) u0[s][c] = u1[s][c] = u2[s][c] = r0[s][c] = r1[s][c] = d0[s][c] = 0;

    // LDS ring slot of local plane q (q3 = q % 3) for a population with march-axis component cz
    auto slot = [](int cz, int q, int q3) {
        if (K == 2) return cz > 0 ? (q & 3) : cz == 0 ? q3 : (q & 1);
        return cz > 0 ? q3 : cz == 0 ? (q & 1) : 0;
    };

    // One iteration pl: stage s computes local plane l = pl - (s - 1).  Stage 1 uses the loads
    // in cur and then issues the loads of plane pl + PF into it; a barrier separates consecutive
    // stages.  With K = 2 a wave that runs ahead into the next iteration's stage 1 writes ring
    // set 1 one plane beyond those the slowest wave may still read in stage 2, so those rings
    // have one slot more than the planes in use.  With K = 3 the next stage 1 (ring set 1) and
    // stage 2 (ring set 2) start only after a barrier that every wave passes once it is done
    // with the stage that reads that set, so the planes in use are enough.
    const int last = seg + 2 * K - 3;  // stage K writes the segment's seg planes
    // first population of the prefetch chunk issued in stage s (chunk(K + 1) = Q)
    auto chunk = [](int s) { return i0 + (Q - i0) * (s - 1) / K; };
    // on = false: a pass past the segment's last plane (see the loop below): its stores go out of
    // range, its other work is never used
    auto body = [&](int pl, Loaded &cur, bool on) {
        const unsigned out_bytes = on ? plane_bytes : 0u;
#pragma unroll
        for (int s = 1; s <= K; ++s) {
            if (s > 1) load_plane(pl + PF, cur, pl + PF <= last, chunk(s), chunk(s + 1));
            const int l = pl - (s - 1);
            if (l >= s - 1) {
                const int l3 = l % 3;
                const int lm3 = (l + 2) % 3;  // (l - 1) % 3
                const int lp3 = (l + 1) % 3;  // (l + 1) % 3
                // stage 1's interior inputs: in 3D the pair's own two elements, the x-neighbour
                // beyond it from the neighbouring lane (DPP, all lanes active here) or, for the
                // first and last pair of a row, from its own extra element
                CT in1[PAIR ? NJ : 1][Q];
                if (PAIR && s == 1) {
#pragma unroll
                    for (int i = i0; i < Q; ++i) {
                        if constexpr (PAIR) {
                            const CT a = dec_loaded<ST, RAW>(cur.pr[i].x), bb = dec_loaded<ST, RAW>(cur.pr[i].y);
                            if (F::kx(i) == 0) {
                                in1[0][i] = a;
                                in1[1][i] = bb;
                            } else if (F::kx(i) > 0) {  // pulls from x - 1
                                const CT left = dpp_move<kDppWaveShr1>(bb);
                                const CT edge = dec_loaded<ST, RAW>(cur.fx1[i]);  // decoded on every lane: a select,
                                in1[0][i] = row_first ? edge : left;             // not a branch
                                in1[1][i] = a;
                            } else {  // pulls from x + 1
                                const CT right = dpp_move<kDppWaveShl1>(a);
                                const CT edge = dec_loaded<ST, RAW>(cur.fx1[i]);
                                in1[0][i] = bb;
                                in1[1][i] = row_last ? edge : right;
                            }
                        }
                    }
                }
                CT outK[PAIR ? NJ : 1][Q];  // stage K's results of a pair, stored together after the loop
                const int Zq = z0 - (K - 1) + l;  // stage K: in [z0, z0 + seg)
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    // ring columns work in stages 1 .. K - ring (a slot without a column has ring K)
                    if (c >= NJ && (PAIR ? rbx[c] > K - s : (C::ring_of(c - NJ) > K - s || rbx[c] == K))) continue;
                    CT sv[Q];
                    sv[0] = 0;
                    if (s == 1) {
#pragma unroll
                        for (int i = i0; i < Q; ++i) {
                            if (c >= NJ)
                                sv[i] = dec_loaded<ST, RAW>(cur.rg[c < NJ ? 0 : c - NJ][i]);
                            else if constexpr (PAIR)
                                sv[i] = in1[c < NJ ? c : 0][i];
                            else
                                sv[i] = dec_loaded<ST, RAW>(cur.in[c < NJ ? c : 0][i]);
                        }
                    } else {
                        const int set = s - 1;  // ring set read, in its own coordinates
                        const int xs = cxl[c] - (s - 2), ys = cyl[c] - HY * (s - 2);
#pragma unroll
                        for (int i = i0; i < Q; ++i) {
                            if (F::moves_xy(i)) {
                                const int kz = F::kz(i);
                                const int q = l - kz;
                                const int q3 = kz > 0 ? lm3 : kz < 0 ? lp3 : l3;
                                const RE e = ring[set_off(set) + (F::plane_off(i, K) + slot(kz, q, q3)) * set_pl(set) +
                                                  lidx(set, xs - F::kx(i), ys - F::ky(i))];
                                if constexpr (CARRY)
                                    sv[i] = e;
                                else
                                    sv[i] = dec_io<ST, RAW>(e);
                            } else {
                                sv[i] = i == IU ? u2[set][c] : i == IR ? r1[set][c] : d0[set][c];
                            }
                        }
                    }
                    collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(k, sv);
                    if (s == K) {
                        if constexpr (PAIR) {
                            if (c < NJ)
#pragma unroll
                                for (int i = i0; i < Q; ++i) outK[c < NJ ? c : 0][i] = sv[i];
                        } else if (c < NJ) {
                            // cells outside the box have an out-of-range offset: no branch
#pragma unroll
                            for (int i = i0; i < Q; ++i)
                                buf_store<E>(enc_io<ST, RAW>(sv[i]),
                                             plane_rsrc(dst + (size_t)i * N + (size_t)Zq * plane, out_bytes),
                                             so[c < NJ ? c : 0]);
                        }
                    } else {
                        const int lxy = lidx(s, cxl[c] - (s - 1), cyl[c] - HY * (s - 1));
                        const bool keep_local = c < NJ ? true
                                                : PAIR ? rbx[c] <= K - s - 1 : C::ring_of(c - NJ) <= K - s - 1;
#pragma unroll
                        for (int i = i0; i < Q; ++i) {
                            // as stored and reloaded (FP64, FP32: the value itself), or carried
                            // unrounded (16-bit formats)
                            CT v = sv[i];
                            if constexpr (!CARRY) v = dec_io<ST, RAW>(enc_io<ST, RAW>(sv[i]));
                            if (F::moves_xy(i)) {
                                if constexpr (CARRY)
                                    ring[set_off(s) + (F::plane_off(i, K) + slot(F::kz(i), l, l3)) * set_pl(s) + lxy] = v;
                                else
                                    ring[set_off(s) + (F::plane_off(i, K) + slot(F::kz(i), l, l3)) * set_pl(s) + lxy] =
                                        enc_io<ST, RAW>(sv[i]);
                            } else if (keep_local) {
                                if (i == IU) u0[s][c] = v;
                                if (i == IR) r0[s][c] = v;
                                if (i == ID) d0[s][c] = v;
                            }
                        }
                    }
                }
                if (PAIR && s == K) {
                    // a pair's step t+K: one access per population; a pair outside the box has an
                    // out-of-range offset, so there is no branch
#pragma unroll
                    for (int i = i0; i < Q; ++i) {
                        E2 v;
                        v.x = enc_io<ST, RAW>(outK[0][i]);
                        v.y = enc_io<ST, RAW>(outK[PAIR ? 1 : 0][i]);
                        buf_store2<E>(v, plane_rsrc(dst + (size_t)i * N + (size_t)Zq * plane, out_bytes), so[0]);
                    }
                }
            }
            if (s == 1) {
                // the next loads into `cur` may not move above the last reads of its old values:
                // otherwise the two overlap, the loop latch copies the new values into the old
                // registers, and that copy waits for the loads it was meant to keep in flight
                __builtin_amdgcn_sched_barrier(0);
                load_plane(pl + PF, cur, pl + PF <= last, chunk(1), chunk(2));  // in flight across the stages
            }
            if (s < K) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
            }
        }
#pragma unroll
        for (int s = 1; s < K; ++s)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                u2[s][c] = u1[s][c];
                u1[s][c] = u0[s][c];
                r1[s][c] = r0[s][c];
            }
    };

    load_plane(0, la, true, 0, Q);
    if constexpr (PF == 2) {
        // plane 0's loads must be issued before plane 1's: the loop's first use of plane 0 then
        // waits only for those (issued in the other order, the wait at the loop head, shared by
        // every pass, is for all loads in flight)
        __builtin_amdgcn_sched_barrier(0);
        load_plane(1, lb, true, 0, Q);  // seg >= 1: at least 2K - 1 >= 3 planes
        // every pass through the loop runs both bodies, so there is one path to the loop head
        // and the compiler's wait counts there stay exact (with the second body under a branch it
        // waits for every load in flight); past the last plane the second body stores nothing
        for (int pl = 0; pl <= last; pl += 2) {
            body(pl, la, true);
            body(pl + 1, lb, pl + 1 <= last);
        }
    } else {
        for (int pl = 0; pl <= last; ++pl) body(pl, la, true);
    }
}

}  // namespace lbm
