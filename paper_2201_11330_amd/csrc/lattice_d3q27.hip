// D3Q27 instantiation of the liblbm.so kernels.
#include "impl.hpp"

namespace imexlbm {

const Ops* ops_d3q27(lbm_storage s) { return make_ops<2>(s); }

}  // namespace imexlbm
