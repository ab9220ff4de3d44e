// Stage kernels for f16 vector rows.
#include "search_impl.hpp"

namespace miann {
template hipError_t launch_dt<DT_F16>(int, const StageArgs&, hipStream_t);
}  // namespace miann
