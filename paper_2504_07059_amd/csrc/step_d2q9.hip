// Forward kernels of the D2Q9 lattice (instantiations of step_impl.hpp).
#include "step_impl.hpp"

namespace lbmmc {

template hipError_t launch_step_lat<0>(int, const Launch&);
template hipError_t launch_init_lat<0>(int, const LatParams*, int, const LatParams&,
                                           const double*, const float*, float*, float*,
                                           unsigned*, hipStream_t);
template hipError_t launch_moments_lat<0>(int, const Launch&, int, float*, float*, float*,
                                              float*, float*, double*, int);

}  // namespace lbmmc
