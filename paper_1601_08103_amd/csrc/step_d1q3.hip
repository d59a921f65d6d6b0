// Step launch sequence of the D1Q3 velocity set (explicit instantiation; see step_impl.hpp).
#include "step_impl.hpp"

template lbm_status lbm::api::step_lattice<lbm::VS_D1Q3>(lbm_lee *h, int64_t nsteps, hipStream_t st);
