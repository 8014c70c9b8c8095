// gm_fam_expdisk.hip -- kernels of the model family: exponential disk + sky (7).
#include "gm_launch.h"

namespace gm {
FamilyOps ops_expdisk() { return make_ops<FamSingle<ExpDisk>, 2, 25>(); }
}  // namespace gm
