// Single-precision instantiation of the orbit integrator (compiled with
// contraction of a*b+c into FMA allowed).
#include "integrate_impl.h"

namespace sw {
hipError_t launch_integrate_f32(const IntegrateLaunch& L, hipStream_t st) { return launch_integrate_t<float>(L, st); }
}  // namespace sw
