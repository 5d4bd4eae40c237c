// Transpose kernels of 1-byte elements, single launches (the kernel templates
// are in tpose_dev.hpp; one element size and form per translation unit, so
// the instantiations compile in parallel).
#include "tpose_dev.hpp"

namespace xtr {
namespace tpk {

int launch_single_e1(const void *src, void *dst, int64_t rows, int64_t cols, int64_t ld_src,
                       int64_t ld_dst, hipStream_t stream) {
    return launch_one<1>(src, dst, rows, cols, ld_src, ld_dst, stream);
}

}  // namespace tpk
}  // namespace xtr
