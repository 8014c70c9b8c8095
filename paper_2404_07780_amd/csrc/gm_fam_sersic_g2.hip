// gm_fam_sersic_g2.hip -- kernels of the model family single Sersic + sky (8 LM variables), 2 plane groups; PSF sides 15, 25, 41 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_sersic_2() { return make_variant<FamSersic, 2, 15, 25, 41>(); }
}  // namespace gm
