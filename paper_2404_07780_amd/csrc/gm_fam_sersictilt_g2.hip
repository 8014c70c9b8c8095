// gm_fam_sersictilt_g2.hip -- kernels of the model family single Sersic + tilted-plane sky (10 LM variables), 2 plane groups; PSF sides 15, 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_sersictilt_2() { return make_variant<FamSersicTilt, 2, 15, 25>(); }
}  // namespace gm
