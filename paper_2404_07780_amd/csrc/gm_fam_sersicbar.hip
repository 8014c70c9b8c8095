// gm_fam_sersicbar.hip -- kernels of the model family: Sersic + Ferrer bar, shared centre, + sky (12).
#include "gm_launch.h"

namespace gm {
FamilyOps ops_sersicbar() { return make_ops<FamSersicBar, 3, 25>(); }
}  // namespace gm
