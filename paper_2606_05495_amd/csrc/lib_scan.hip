// The library stage of library-call templates: rocPRIM's device-wide
// inclusive scan, captured into the job graph between the template's own
// begin and end kernels.
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include "kernels.hpp"

namespace setrt {

namespace {
struct WidenI32 {
  __host__ __device__ int64_t operator()(int32_t v) const { return (int64_t)v; }
};
}  // namespace

hipError_t lib_scan(void* ws, size_t& ws_bytes, const int32_t* in, int64_t* out, size_t n, hipStream_t st) {
  auto it = rocprim::make_transform_iterator(in, WidenI32{});
  return rocprim::inclusive_scan(ws, ws_bytes, it, out, n, rocprim::plus<int64_t>(), st, false);
}

}  // namespace setrt
