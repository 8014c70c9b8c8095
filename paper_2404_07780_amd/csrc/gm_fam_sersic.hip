// gm_fam_sersic.hip -- kernels of the model family: single Sersic + sky (8 LM variables); PSF sides 15 and 25 compiled.
#include "gm_launch.h"

namespace gm {
FamilyOps ops_sersic() { return make_ops<FamSersic, 2, 15, 25>(); }
}  // namespace gm
