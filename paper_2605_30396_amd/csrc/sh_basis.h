// Real spherical harmonics of degree 1..3 in Cartesian form (the view-
// dependent SH functions whose coefficients Sec. 2.2 compresses), shared by
// the radiance kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace sc {

constexpr float kShC0 = 0.28209479177387814f;   // degree-0 constant 1 / (2 sqrt(pi))

// Real SH of degree 1..L in Cartesian form, Condon-Shortley phase, m = -l..l.
// Constants are the normalisations sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!),
// times sqrt(2) for m != 0, folded into each polynomial.
template <int NB>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y) {
    const float c1 = 0.48860251190291992f;      // sqrt(3/(4 pi))
    Y[0] = -c1 * y;
    Y[1] = c1 * z;
    Y[2] = -c1 * x;
    if (NB >= 8) {
        const float xx = x * x, yy = y * y, zz = z * z;
        const float c2a = 1.0925484305920792f;  // sqrt(15/(4 pi))
        const float c2b = 0.31539156525252005f; // sqrt(5/(16 pi))
        const float c2c = 0.54627421529603959f; // sqrt(15/(16 pi))
        Y[3] = c2a * x * y;
        Y[4] = -c2a * y * z;
        Y[5] = c2b * (2.f * zz - xx - yy);
        Y[6] = -c2a * x * z;
        Y[7] = c2c * (xx - yy);
        if (NB >= 15) {
            const float c3a = 0.59004358992664352f;  // sqrt(35/(32 pi))
            const float c3b = 2.8906114426405538f;   // sqrt(105/(4 pi))
            const float c3c = 0.45704579946446572f;  // sqrt(21/(32 pi))
            const float c3d = 0.37317633259011540f;  // sqrt(7/(16 pi))
            const float c3e = 1.4453057213202769f;   // sqrt(105/(16 pi))
            Y[8] = -c3a * y * (3.f * xx - yy);
            Y[9] = c3b * x * y * z;
            Y[10] = -c3c * y * (4.f * zz - xx - yy);
            Y[11] = c3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
            Y[12] = -c3c * x * (4.f * zz - xx - yy);
            Y[13] = c3e * z * (xx - yy);
            Y[14] = -c3a * x * (xx - 3.f * yy);
        }
    }
}

}  // namespace sc
