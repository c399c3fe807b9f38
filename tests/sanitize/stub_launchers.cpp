// Host-only stand-ins for the device-side functions of the library, so its
// host engine can be built with g++ and the address / undefined-behaviour
// sanitizers and exercised on a machine without a GPU.  Every stand-in
// reports that no device is present; the host logic under test (argument
// checks, geometry, tile rules, the connectivity flood fill) never reaches
// them.
#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

#include "pcg_types.h"

namespace pcgmi {
hipError_t launch_iter(int, int, int, int, const BatchHeader *, const Slot *, hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_classify(const double *, uint8_t *, int64_t, int, unsigned long long *,
                           hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_encode(const double *, const uint8_t *, double *, float *, int64_t, int *,
                         hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_copy(const double *, double *, size_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_pack_mask(const uint8_t *, uint32_t *, int, int, int64_t, hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_triad(double *, const double *, const double *, double, size_t, hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_check_frac(const double *, const double *, const double *, const double *,
                             const double *, int64_t, int64_t, int64_t, int64_t, int *,
                             hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_project(const Slot *, const double *, double, double, const double *const[3],
                          const double *const[3], double *const[3], int, hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_rhs(const Slot *, double, double, const double *const[3],
                      const double *const[3], double *, int, hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t launch_divnorm(const Slot *, double, const double *, const double *, const double *,
                          double *, int, hipStream_t)
{
    return hipErrorNoDevice;
}
hipError_t static_scratch(void **, size_t *) { return hipErrorNoDevice; }
}  // namespace pcgmi
