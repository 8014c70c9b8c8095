// gm_fam_sersicbar_g3.hip -- kernels of the model family Sersic + Ferrer bar with a shared centre + sky (12 LM variables), 3 plane groups; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_sersicbar_3() { return make_variant<FamSersicBar, 3, 25>(); }
}  // namespace gm
