// gm_fam_bulgedisk.hip -- kernels of the model family: Sersic bulge + exponential disk, shared centre, + sky (12).
#include "gm_launch.h"

namespace gm {
FamilyOps ops_bulgedisk() { return make_ops<FamBulgeDisk, 3, 25>(); }
}  // namespace gm
