// gm_fam_sersicbox_g1.hip -- kernels of the model family single boxy Sersic + sky (9 LM variables), 1 plane group; PSF sides 15, 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_sersicbox_1() { return make_variant<FamSersicBox, 1, 15, 25>(); }
}  // namespace gm
