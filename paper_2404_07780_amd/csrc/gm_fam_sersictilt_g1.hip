// gm_fam_sersictilt_g1.hip -- kernels of the model family single Sersic + tilted-plane sky (10 LM variables), 1 plane group; PSF sides 15, 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_sersictilt_1() { return make_variant<FamSersicTilt, 1, 15, 25>(); }
}  // namespace gm
