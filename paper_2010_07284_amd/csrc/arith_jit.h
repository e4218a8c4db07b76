// arith_jit.h -- arithmetic atoms compiled into straight-line kernels (hipRTC).
#pragma once

#include <string>

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace vlg {

// The HIP source of the kernel that evaluates the programs of `a` on pixels
// of type dtype (0 float32, 1 uint8, 2 uint16); "" when a program is not a
// well-formed postfix program within the group limits.  The source does not
// depend on a.out.
std::string arith_jit_source(const ArithGroup &a, int dtype);

// The compiled kernel of arith_jit_source on `device`, compiled on first use
// and kept (with its module) until the process ends; a group that does not
// compile is remembered too.  nullptr on failure (err, if given, says why).
// Thread-safe.  Loads a module: call it before, not during, stream capture.
hipFunction_t arith_jit_function(int device, const ArithGroup &a, int dtype, std::string *err);

// Launch a compiled kernel on the same grid as launch_arith.
hipError_t launch_arith_jit(hipFunction_t fn, hipStream_t s, const Geo &g, const void *img, int64_t chan_elems,
                            const ArithGroup &a, const float *pct);

}  // namespace vlg
