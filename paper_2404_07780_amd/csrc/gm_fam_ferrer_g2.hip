// gm_fam_ferrer_g2.hip -- kernels of the model family Ferrer + sky, 2 plane groups; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_ferrer_2() { return make_variant<FamSingle<Ferrer>, 2, 25>(); }
}  // namespace gm
