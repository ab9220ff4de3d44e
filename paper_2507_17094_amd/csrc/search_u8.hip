// Stage kernels for u8 vector rows.
#include "search_impl.hpp"

namespace miann {
template hipError_t launch_dt<DT_U8>(int, const StageArgs&, hipStream_t);
}  // namespace miann
