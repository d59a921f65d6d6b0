// Step launch sequence of the D3Q27 velocity set (explicit instantiation; see step_impl.hpp).
#include "step_impl.hpp"

template lbm_status lbm::api::step_lattice<lbm::VS_D3Q27>(lbm_lee *h, int64_t nsteps, hipStream_t st);
