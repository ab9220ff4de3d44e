// Stage kernels for f32 vector rows.
#include "search_impl.hpp"

namespace miann {
template hipError_t launch_dt<DT_F32>(int, const StageArgs&, hipStream_t);
}  // namespace miann
