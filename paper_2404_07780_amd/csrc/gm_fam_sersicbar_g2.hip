// gm_fam_sersicbar_g2.hip -- kernels of the model family Sersic + Ferrer bar with a shared centre + sky (12 LM variables), 2 plane groups; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_sersicbar_2() { return make_variant<FamSersicBar, 2, 25>(); }
}  // namespace gm
