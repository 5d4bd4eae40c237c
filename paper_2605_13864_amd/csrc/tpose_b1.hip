// Transpose kernels of 1-byte elements, batched launches (the kernel templates
// are in tpose_dev.hpp; one element size and form per translation unit, so
// the instantiations compile in parallel).
#include "tpose_dev.hpp"

namespace xtr {
namespace tpk {

void launch_group_e1(int w, bool off32, bool lines, int geo, int64_t grid, hipStream_t st,
                       const Job *jobs, const int64_t *bases, int nj, int64_t ntiles,
                       const JobPack *pk, uint32_t *ctr) {
    launch_batched<1>(w, off32, lines, geo, grid, st, jobs, bases, nj, ntiles, pk, ctr);
}

}  // namespace tpk
}  // namespace xtr
