// gm_fam_sersic_g1.hip -- kernels of the model family single Sersic + sky (8 LM variables), 1 plane group; PSF sides 15, 25, 41 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_sersic_1() { return make_variant<FamSersic, 1, 15, 25, 41>(); }
}  // namespace gm
