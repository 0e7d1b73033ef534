// Launcher of the axisymmetric 2D step (kern_axisym.hip).  Not part of the
// public ABI.
#pragma once

#include "acm_internal.h"

namespace acm {

// One axisymmetric single-phase step (x axial, y radial, axis on the -y
// face); tile codes 1 32x8, 2 64x8, 4 64x4, else 32x16.
template <typename T>
hipError_t launch_axisym2d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile, hipStream_t s);

// One axisymmetric two-phase step (kern_twophase.hip); tile codes as for the
// planar two-phase step.
template <typename T>
hipError_t launch_twophase_axisym2d(const Coef<T>& c, const State<T>& in, const State<T>& out, int tile,
                                    hipStream_t s);

}  // namespace acm
