// Stage kernels for fp8 vector rows.
#include "search_impl.hpp"

namespace miann {
template hipError_t launch_dt<DT_FP8>(int, const StageArgs&, hipStream_t);
}  // namespace miann
