// Launch geometry of the empirical-moment kernels (srmra_moments.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace srmra {

struct MomentsGeom {
    int P = 0, T = 0, npairs = 0, S = 0, S1 = 0;   // pixels, tiles per edge, tile pairs, chunks
    int64_t chunk = 0, chunk1 = 0;                 // observations per chunk (M2, M1)
    size_t o_part = 0, o_part1 = 0, total = 0;     // workspace layout
};

MomentsGeom moments_geom(int64_t N, int Ll, int cus);
hipError_t launch_moments(const float* y, int64_t N, int Ll, double* m1, double* m2, void* ws,
                          const MomentsGeom& g, hipStream_t s);

}  // namespace srmra
