// gm_fam_expdisk_g1.hip -- kernels of the model family exponential disk + sky, 1 plane group; PSF side 25 compiled, any other odd side generic.
#include "gm_launch.h"

namespace gm {
Variant var_expdisk_1() { return make_variant<FamSingle<ExpDisk>, 1, 25>(); }
}  // namespace gm
