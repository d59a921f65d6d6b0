// Host-side FP64 coefficient setup (velocity sets, weights, equilibrium coefficients).
//
// Sources in the paper:
//  * monoatomic equilibrium (Section "Derivation of Finite Discrete Velocity Models for
//    Monoatomic Gases"): g_i^eq = f*_i (rho'/rho0 + c_i.u'/theta0
//    + theta' (|c_i|^2 / (2 theta0^2) - D / (2 theta0))), i.e. the polyatomic ansatz with
//    a1 = 1/rho0, a2 = -D/(2 theta0), b = 1/theta0, c1 = 0, c2 = 1/theta0^2, beta = 0, and the
//    adiabatic exponent gamma = (M+2)/M with M = D degrees of freedom;
//  * D1Q3 and D2Q5 weights: subsections "D1Q3" and "D2Q5 for Monoatomic Gases";
//  * the 3D family f*(rho0, theta0, alpha) of Section "3D" (rest, axis, edge, corner weights),
//    with the (theta0, alpha) choices that reduce it to D3Q7, D3Q9, D3Q13 and D3Q19, and the
//    member theta0 = 1/3, alpha = 1/216 with all 27 weights positive (D3Q27);
//  * diatomic D2Q5 and D3Q7 (subsection "D2Q5 for Diatomic Gases" and the "Diatomic Gases"
//    subsection of Section "3D"): printed weights, beta and coefficients, gamma = (M+2)/M with
//    M = 2D - 1.
//  * D2Q9 is derived, not printed: weights w_rest = 1 - 3 theta0 + 4 theta0^2,
//    w_axis = theta0 (1 - 2 theta0), w_diag = theta0 (4 theta0 - 1) / 4 satisfy the similarity
//    conditions of the monoatomic FDVM section in 2D; theta0 = 1/3 gives 4/9, 1/9, 1/36.
#include "tables.hpp"

#include <cstring>

#include "../../include/lbm_lee.h"

namespace lbm {
namespace {

template <class VS>
void copy_velocities(LatticeTable *t) {
    t->D = VS::D;
    t->Q = VS::Q;
    for (int i = 0; i < VS::Q; ++i)
        for (int a = 0; a < 3; ++a) t->c[i][a] = VS::c[i][a];
}

int nonzeros(const int *c) { return (c[0] != 0) + (c[1] != 0) + (c[2] != 0); }

void monoatomic(LatticeTable *t, double rho0, double theta0) {
    t->rho0 = rho0;
    t->theta0 = theta0;
    t->gamma = (t->D + 2.0) / t->D;
    t->a1 = 1.0 / rho0;
    t->a2 = -t->D / (2.0 * theta0);
    t->b = 1.0 / theta0;
    t->c1 = 0.0;
    t->c2 = 1.0 / (theta0 * theta0);
    for (int i = 0; i < t->Q; ++i) t->beta[i] = 0.0;
}

// Weights by number of non-zero velocity components: {rest, axis, edge, corner}.
void weights_by_class(LatticeTable *t, const double w[4]) {
    for (int i = 0; i < t->Q; ++i) t->f[i] = w[nonzeros(t->c[i])];
}

void family3d(LatticeTable *t, double rho0, double theta0, double alpha) {
    const double w[4] = {
        0.5 * rho0 * theta0 * (15.0 * theta0 - 9.0) + rho0 - 8.0 * alpha,
        0.5 * rho0 * theta0 * (2.0 - 5.0 * theta0) + 4.0 * alpha,
        0.125 * rho0 * theta0 * (5.0 * theta0 - 1.0) - 2.0 * alpha,
        alpha,
    };
    weights_by_class(t, w);
    monoatomic(t, rho0, theta0);
}

}  // namespace

bool build_lattice(int id, LatticeTable *t) {
    std::memset(t, 0, sizeof(*t));
    t->id = id;
    switch (id) {
        case LBM_D1Q3: {
            copy_velocities<VS_D1Q3>(t);
            const double w[4] = {2.0 / 3.0, 1.0 / 6.0, 0.0, 0.0};
            weights_by_class(t, w);
            monoatomic(t, 1.0, 1.0 / 3.0);
            t->name = "D1Q3";
            return true;
        }
        case LBM_D2Q5: {
            copy_velocities<VS_D2Q5>(t);
            const double w[4] = {0.5, 0.125, 0.0, 0.0};
            weights_by_class(t, w);
            monoatomic(t, 1.0, 0.25);
            t->name = "D2Q5";
            return true;
        }
        case LBM_D2Q9: {
            copy_velocities<VS_D2Q9>(t);
            const double th = 1.0 / 3.0;
            const double w[4] = {1.0 - 3.0 * th + 4.0 * th * th, th * (1.0 - 2.0 * th), th * (4.0 * th - 1.0) / 4.0, 0.0};
            weights_by_class(t, w);
            monoatomic(t, 1.0, th);
            t->name = "D2Q9";
            return true;
        }
        case LBM_D3Q7:
            copy_velocities<VS_D3Q7>(t);
            family3d(t, 1.0, 0.2, 0.0);
            t->name = "D3Q7";
            return true;
        case LBM_D3Q9:
            copy_velocities<VS_D3Q9>(t);
            family3d(t, 1.0, 0.6, 3.0 / 40.0);
            t->name = "D3Q9";
            return true;
        case LBM_D3Q13:
            copy_velocities<VS_D3Q13>(t);
            family3d(t, 1.0, 0.4, 0.0);
            t->name = "D3Q13";
            return true;
        case LBM_D3Q19:
            copy_velocities<VS_D3Q19>(t);
            family3d(t, 1.0, 0.3, 0.0);
            t->name = "D3Q19";
            return true;
        case LBM_D3Q27:
            // a member of the family with every weight positive: theta0 = 1/3, alpha = 1/216 gives
            // 8/27, 2/27, 1/54, 1/216 (the products of the D1Q3 weights 2/3, 1/6, 1/6)
            copy_velocities<VS_D3Q27>(t);
            family3d(t, 1.0, 1.0 / 3.0, 1.0 / 216.0);
            t->name = "D3Q27";
            return true;
        case LBM_D2Q5_DIA: {
            copy_velocities<VS_D2Q5>(t);
            const double w[4] = {8.0 / 3.0, 1.0, 0.0, 0.0};
            weights_by_class(t, w);
            t->rho0 = 20.0 / 3.0;
            t->theta0 = 0.3;
            t->gamma = 5.0 / 3.0;  // M = 2D - 1 = 3
            t->a1 = 1.0 / t->rho0;
            t->a2 = -5.0;
            t->b = 1.0 / t->theta0;
            t->c1 = 0.0;
            t->c2 = 5.0 / t->theta0;
            for (int i = 0; i < t->Q; ++i) t->beta[i] = nonzeros(t->c[i]) ? 0.5 : 0.0;
            t->name = "D2Q5_DIA";
            return true;
        }
        case LBM_D3Q7_DIA: {
            copy_velocities<VS_D3Q7>(t);
            const double f1 = 5.0 / 42.0;  // the member of the family whose Gamma(k) is unitary
            const double w[4] = {12.0 / 5.0 * f1, f1, 0.0, 0.0};
            weights_by_class(t, w);
            t->rho0 = 42.0 / 5.0 * f1;
            t->theta0 = 5.0 / 21.0;
            t->gamma = 7.0 / 5.0;  // M = 2D - 1 = 5
            t->a1 = 1.0 / t->rho0;
            t->a2 = -21.0 / 2.0;
            t->b = 21.0 / 5.0;
            t->c1 = 0.0;
            t->c2 = 147.0 / 5.0;
            for (int i = 0; i < t->Q; ++i) t->beta[i] = nonzeros(t->c[i]) ? 2.0 / 3.0 : 0.0;
            t->name = "D3Q7_DIA";
            return true;
        }
        default:
            return false;
    }
}

}  // namespace lbm
