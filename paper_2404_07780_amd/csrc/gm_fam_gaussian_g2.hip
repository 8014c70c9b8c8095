// gm_fam_gaussian_g2.hip -- kernels of the model family Gaussian + sky, 2 plane groups; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_gaussian_2() { return make_variant<FamSingle<Gaussian>, 2, 25>(); }
}  // namespace gm
