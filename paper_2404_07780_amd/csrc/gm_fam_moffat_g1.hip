// gm_fam_moffat_g1.hip -- kernels of the model family Moffat + sky, 1 plane group; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_moffat_1() { return make_variant<FamSingle<Moffat>, 1, 25>(); }
}  // namespace gm
