// D3Q19 instantiation of the liblbm.so kernels.
#include "impl.hpp"

namespace imexlbm {

const Ops* ops_d3q19(lbm_storage s) { return make_ops<1>(s); }

}  // namespace imexlbm
