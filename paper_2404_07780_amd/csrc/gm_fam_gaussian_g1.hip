// gm_fam_gaussian_g1.hip -- kernels of the model family Gaussian + sky, 1 plane group; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_gaussian_1() { return make_variant<FamSingle<Gaussian>, 1, 25>(); }
}  // namespace gm
