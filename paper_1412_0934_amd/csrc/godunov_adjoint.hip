// Reverse-mode adjoint of the Godunov step (gfx950).
#include "godunov_internal.h"

namespace gd {

int launch_adjoint(int, int, const PatchDesc &, const double *, const double *, const double *,
                   double *, const Scalars &, double, hipStream_t)
{
    return (int)hipErrorNotSupported;
}

}  // namespace gd
