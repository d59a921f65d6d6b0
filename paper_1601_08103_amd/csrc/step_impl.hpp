// The step launch sequence of one velocity set: the K-step, one-step, in-place and open-box
// kernels for every storage type.  Instantiated once per velocity set, in its own translation
// unit (step_<set>.hip), so the library compiles in parallel.
#pragma once

#include "internal.hpp"

namespace lbm {
namespace api {

template <class VSet>
lbm_status step_lattice(lbm_lee *h, int64_t nsteps, hipStream_t st) {
    const int variant = resolve_variant(h);
    const int bc = h->desc.bc;
    return visit_storage<VSet>(h->desc.storage, [&](auto vs, auto sto) -> lbm_status {
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
            if (sponge_layer(&h->desc)) {  // the largest slab: depth W times a full face
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
            // one block per resident slot (each block stages the weights once, then its waves walk
            // the tiles), at most one per four tiles
            long long slots = 4096;
            if constexpr (NetGeom<VS>::fits) {
                int per_cu = 0;
                if (h->cus > 0 &&
                    hipOccupancyMaxActiveBlocksPerMultiprocessor(
                        &per_cu, (const void *)&ghost_mlp_kernel<VS, ST, true>, 256, 0) == hipSuccess &&
                    per_cu > 0)
                    slots = (long long)per_cu * h->cus;
                (void)hipGetLastError();
            }
            ghost_blocks = (tune & LBM_TUNE_NET_ONE_BLOCK) ? 1u : (unsigned)std::min<long long>((tiles + 3) / 4, slots);
        }
        auto run = [&](auto skip, auto half) -> lbm_status {
            constexpr bool SK = decltype(skip)::value;
            constexpr bool HF = decltype(half)::value;
            const bool dpp = variant == LBM_VARIANT_DPP || variant == LBM_VARIANT_DPP2;
            const unsigned g_dpp4t = dpp && vec == 4 && fullrow ? dpp_grid((const void *)&step_dpp<VS, ST, 4, true, SK, HF>) : 1;
            const unsigned g_dpp4f = dpp && vec == 4 && !fullrow ? dpp_grid((const void *)&step_dpp<VS, ST, 4, false, SK, HF>) : 1;
            const unsigned g_dpp2t = dpp && vec == 2 && fullrow ? dpp_grid((const void *)&step_dpp<VS, ST, 2, true, SK, HF>) : 1;
            const unsigned g_dpp2f = dpp && vec == 2 && !fullrow ? dpp_grid((const void *)&step_dpp<VS, ST, 2, false, SK, HF>) : 1;
            // 3D open boxes with the DPP bulk step close their x faces in the bulk kernel (not
            // with the network on the helper stream: the bulk kernel reads this step's ghosts)
            const bool bulk_x = VS::D == 3 && dpp && bc != LBM_BC_PERIODIC && !(bc == LBM_BC_MLP && fork);
            // with bulk_x a sponge layer is damped by the bulk and shell kernels as they store; not
            // for storage with a raw step domain (E3M12), whose damping (a real-domain decode and
            // encode per value) takes the bulk kernel to 132 registers: slower than a sponge pass
            const int layer_w = bulk_x && sponge_layer(&h->desc) && !ST::has_raw ? h->desc.sponge_width : 0;
            auto open_bulk = [&](const E *src, E *dst) {
                if constexpr (VS::D == 3) {
                    auto go = [&](auto kern) {
                        kern<<<dpp_grid((const void *)kern), 256, 0, st>>>(src, dst, h->nx, h->ny, h->nz, h->N, cpr,
                                                                           waves, tune, k, bc, h->ghost, ft, fk,
                                                                           layer_w, h->desc.sponge_sigma);
                    };
                    auto pick = [&](auto layer) {
                        constexpr bool LY = decltype(layer)::value;
                        if (vec == 4)
                            fullrow ? go(&step_dpp_open<VS, ST, 4, true, SK, HF, LY>)
                                    : go(&step_dpp_open<VS, ST, 4, false, SK, HF, LY>);
                        else
                            fullrow ? go(&step_dpp_open<VS, ST, 2, true, SK, HF, LY>)
                                    : go(&step_dpp_open<VS, ST, 2, false, SK, HF, LY>);
                    };
                    if constexpr (!ST::has_raw) {
                        if (layer_w > 0) {
                            pick(std::true_type{});
                            return;
                        }
                    }
                    pick(std::false_type{});
                }
            };
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
                        const long long tiles_x = (fx + SH::TX - 1) / SH::TX, tiles_y = (fy + SH::TY - 1) / SH::TY;
                        auto fn = step_tbk<VS, ST, SK, HF, K, SH::TX, SH::TY, SH::NT, SH::WPE>;
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
            if (variant == LBM_VARIANT_RESIDENT) {
                if (nsteps <= 0) return LBM_OK;
                const E *src = static_cast<const E *>(h->buf[h->cur]);
                E *dst = static_cast<E *>(h->buf[h->cur ^ (int)(nsteps & 1)]);
                const size_t lds = 2 * (size_t)VS::Q * h->N * sizeof(E);
                // more than 64 KiB of dynamic LDS has to be allowed per kernel
                LBM_HIP(hipFuncSetAttribute((const void *)&step_resident<VS, ST, SK, HF>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kResidentLds));
                step_resident<VS, ST, SK, HF><<<1, 1024, lds, st>>>(src, dst, h->nx, h->ny, h->nz, (int)h->N, nsteps, k);
                lbm_status ls = launch_check();
                if (ls != LBM_OK) return ls;
                h->cur ^= (int)(nsteps & 1);
                h->steps += nsteps;
                return LBM_OK;
            }
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
                            // a sponge layer behind the network (width 0: none) is damped inside the step kernel
                            open_step_2d<VS, ST, SK, HF, true><<<face_blocks + bulk_blocks, 256, 0, st>>>(
                                src, dst, h->N, bc, (int)face_blocks, h->net, h->ghost, hin, hout, ft, k, ks, fk,
                                h->desc.sponge_width, h->desc.sponge_sigma);
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
                    if constexpr (NetGeom<VS>::fits) {
                        if (hin)
                            ghost_mlp_kernel<VS, ST, true><<<ghost_blocks, 256, 0, fork ? h->aux : st>>>(
                                src, h->N, h->net, h->ghost, hin, hout, ft, fk);
                        else
                            ghost_mlp_kernel<VS, ST, false><<<ghost_blocks, 256, 0, fork ? h->aux : st>>>(
                                src, h->N, h->net, h->ghost, hin, hout, ft, fk);
                    }
                    if (fork) LBM_HIP(hipEventRecord(h->join, h->aux));
                    h->hist_valid = true;
                }
                if (bulk_x) {
                    open_bulk(src, dst);
                } else if (variant == LBM_VARIANT_GENERIC) {
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
                    shell_kernel<VS, ST, SK, HF><<<dim3(shell_x, 2 * VS::D - (bulk_x ? 2 : 0)), 256, 0, st>>>(
                        src, dst, h->N, bc, h->ghost, ft, ks, fk, bulk_x ? 1 : 0, layer_w, h->desc.sponge_sigma);
                    if (sponge_layer(&h->desc) && layer_w == 0)
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
}

}  // namespace api
}  // namespace lbm
