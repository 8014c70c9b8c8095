// gm_fam_sersicbox_g2.hip -- kernels of the model family single boxy Sersic + sky (9 LM variables), 2 plane groups; PSF sides 15, 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_sersicbox_2() { return make_variant<FamSersicBox, 2, 15, 25>(); }
}  // namespace gm
