/* Lorenzo-predictor quantizer used only to synthesise decompressed test inputs.
 *
 * It stands in for an SZ-style base compressor: each value is predicted from
 * already reconstructed neighbours with the 3D (7-point) Lorenzo stencil,
 * the residual is quantised with bin width 2*eps (mid-tread, ties to even) and
 * the reconstruction p + 2*eps*q is stored.  Out-of-domain neighbours count as
 * zero.  Everything is computed in double; the caller casts to the field type.
 * The errors this produces are spatially correlated, unlike a plain uniform
 * quantiser.
 */
#include <math.h>
#include <stdint.h>

void synth_lorenzo3d(const double *f, double *out, int64_t nx, int64_t ny,
                     int64_t nz, double eps) {
  const double bin = 2.0 * eps;
  const int64_t sy = nx, sz = nx * ny;
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t i = x + sy * y + sz * z;
#define R(dx, dy, dz)                                                          \
  ((x - (dx) >= 0 && y - (dy) >= 0 && z - (dz) >= 0)                           \
       ? out[i - (dx) - sy * (dy) - sz * (dz)]                                 \
       : 0.0)
        const double p = R(1, 0, 0) + R(0, 1, 0) + R(0, 0, 1) - R(1, 1, 0) -
                         R(1, 0, 1) - R(0, 1, 1) + R(1, 1, 1);
#undef R
        const double q = nearbyint((f[i] - p) / bin);
        out[i] = p + bin * q;
      }
}
