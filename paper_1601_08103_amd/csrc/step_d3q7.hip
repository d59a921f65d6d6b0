// Step launch sequence of the D3Q7 velocity set (explicit instantiation; see step_impl.hpp).
#include "step_impl.hpp"

template lbm_status lbm::api::step_lattice<lbm::VS_D3Q7>(lbm_lee *h, int64_t nsteps, hipStream_t st);
