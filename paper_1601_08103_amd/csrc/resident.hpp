// Whole-box steps in one launch for periodic boxes small enough to live in LDS (two copies of
// the state within 160 KiB, a CU's LDS): one block of 1024 threads loads the state, runs every step out of
// LDS with a block barrier between steps, and stores the result.  A tiny box (the paper's 1D
// runs, small convergence-study grids) is otherwise bound by one kernel launch per step.  The
// arithmetic is step_generic's, value for value: the same gathers, collision, and rounding to
// the storage format after every step.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace lbm {

constexpr size_t kResidentLds = 160 * 1024;  // bytes: both copies of the state (dynamic LDS)

template <class VS, class ST, bool SKIP0, bool HALF>
__global__ __launch_bounds__(1024) void step_resident(const typename ST::elem *__restrict__ src,
                                                      typename ST::elem *__restrict__ dst, int nx, int ny, int nz,
                                                      int N, long long nsteps, StepCoef<typename ST::comp, VS::Q> k) {
    using CT = typename ST::comp;
    using E = typename ST::elem;
    extern __shared__ __align__(16) unsigned char resident_lds[];
    E *A = reinterpret_cast<E *>(resident_lds);
    E *B = A + (size_t)VS::Q * N;
    const int QN = VS::Q * N;
    // both copies start as the state (the rest population, when the step leaves it out, keeps it)
    for (int t = threadIdx.x; t < QN; t += blockDim.x) {
        const E v = src[t];
        A[t] = v;
        B[t] = v;
    }
    __syncthreads();
    for (long long step = 0; step < nsteps; ++step) {
        for (int cell = threadIdx.x; cell < N; cell += blockDim.x) {
            const int x = cell % nx;
            const int r = cell / nx;
            const int y = r % ny;
            const int z = r / ny;
            CT s[VS::Q];
            s[0] = 0;
#pragma unroll
            for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) {
                const int xs = wrap_add(x, -VS::cx(i), nx);
                const int ys = wrap_add(y, -VS::cy(i), ny);
                const int zs = wrap_add(z, -VS::cz(i), nz);
                s[i] = dec_io<ST, ST::has_raw>(A[i * N + (zs * ny + ys) * nx + xs]);
            }
            collide<VS, CT, split_constants<ST>(), SKIP0, HALF>(k, s);
#pragma unroll
            for (int i = SKIP0 ? 1 : 0; i < VS::Q; ++i) B[i * N + cell] = enc_io<ST, ST::has_raw>(s[i]);
        }
        __syncthreads();
        E *tmp = A;
        A = B;
        B = tmp;
    }
    for (int t = threadIdx.x; t < QN; t += blockDim.x) dst[t] = A[t];
}

}  // namespace lbm
