// gm_fam_ferrer_g1.hip -- kernels of the model family Ferrer + sky, 1 plane group; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_ferrer_1() { return make_variant<FamSingle<Ferrer>, 1, 25>(); }
}  // namespace gm
