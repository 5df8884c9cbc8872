// Double-precision instantiation of the orbit integrator.  This translation
// unit is compiled with -ffp-contract=off: every expression is evaluated in
// the order written, with IEEE square root and division, so that the
// trajectories are reproducible to the last bit.
#include "integrate_impl.h"

namespace sw {
hipError_t launch_integrate_f64(const IntegrateLaunch& L, hipStream_t st) { return launch_integrate_t<double>(L, st); }
}  // namespace sw
