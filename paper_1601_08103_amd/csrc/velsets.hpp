// Compile-time velocity sets of the LEE lattice Boltzmann schemes.
//
// Velocities of Section "Examples of Velocity Sets": D1Q3, D2Q5, the 27-velocity 3D family
// (in full as D3Q27, and reduced to D3Q7 / D3Q9 / D3Q13 / D3Q19 by its zero weights), and D2Q9
// (rest, axes and diagonals; not in the paper).  The diatomic D2Q5/D3Q7 sets use the same velocities as
// their monoatomic twins and differ only in the runtime coefficient table.
//
// Canonical order: rest, -x, +x, -y, +y, -z, +z, then edges grouped by the plane they lie in
// (xy, xz, yz) with sign patterns in lexicographic order, then corners in lexicographic order.
#pragma once

namespace lbm {

template <int D_, int Q_>
struct VelSetBase {
    static constexpr int D = D_;
    static constexpr int Q = Q_;
};

// REST0: the set has a rest velocity at index 0 that the collision may leave untouched (this
// is decided per coefficient table on the host; sets whose rest population is always coupled
// are compiled without the rest-skipping kernels).
#define LBM_VELSET(NAME, D_, Q_, REST0, ...)                                            \
    struct NAME : VelSetBase<D_, Q_> {                                                  \
        static constexpr bool rest_may_decouple = REST0;                                \
        static constexpr signed char c[Q_][3] = {__VA_ARGS__};                          \
        static constexpr int cx(int i) { return c[i][0]; }                              \
        static constexpr int cy(int i) { return c[i][1]; }                              \
        static constexpr int cz(int i) { return c[i][2]; }                              \
        static constexpr int c2(int i) { return cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i); } \
    };

LBM_VELSET(VS_D1Q3, 1, 3, true, {0, 0, 0}, {-1, 0, 0}, {1, 0, 0})

LBM_VELSET(VS_D2Q5, 2, 5, true, {0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0})

LBM_VELSET(VS_D2Q9, 2, 9, false, {0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0},
           {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}, {1, 1, 0})

LBM_VELSET(VS_D3Q7, 3, 7, true, {0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1})

LBM_VELSET(VS_D3Q9, 3, 9, true, {0, 0, 0}, {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1},
           {1, -1, -1}, {1, -1, 1}, {1, 1, -1}, {1, 1, 1})

LBM_VELSET(VS_D3Q13, 3, 13, true, {0, 0, 0},
           {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}, {1, 1, 0},
           {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1}, {1, 0, 1},
           {0, -1, -1}, {0, -1, 1}, {0, 1, -1}, {0, 1, 1})

LBM_VELSET(VS_D3Q19, 3, 19, false, {0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1},
           {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}, {1, 1, 0},
           {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1}, {1, 0, 1},
           {0, -1, -1}, {0, -1, 1}, {0, 1, -1}, {0, 1, 1})

// The full 27-velocity member of the 3D family (every weight positive for alpha > 0).
LBM_VELSET(VS_D3Q27, 3, 27, false, {0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1},
           {-1, -1, 0}, {-1, 1, 0}, {1, -1, 0}, {1, 1, 0},
           {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1}, {1, 0, 1},
           {0, -1, -1}, {0, -1, 1}, {0, 1, -1}, {0, 1, 1},
           {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1},
           {1, -1, -1}, {1, -1, 1}, {1, 1, -1}, {1, 1, 1})

#undef LBM_VELSET

constexpr int kMaxQ = 27;

}  // namespace lbm
