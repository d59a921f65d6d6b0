// Host-side FP64 coefficient setup of the LEE lattice Boltzmann schemes.
#pragma once

#include "velsets.hpp"

namespace lbm {

struct LatticeTable {
    int id;
    int D, Q;
    int c[kMaxQ][3];
    double f[kMaxQ];     // weights f*_i
    double beta[kMaxQ];  // extra energies beta_i
    double rho0, theta0, gamma;
    double a1, a2, b, c1, c2;  // equilibrium coefficients of the polyatomic ansatz
    const char *name;
};

// Fill `t` for lattice id (LBM_D1Q3 ...).  Returns false for an unknown id.
bool build_lattice(int id, LatticeTable *t);

}  // namespace lbm
