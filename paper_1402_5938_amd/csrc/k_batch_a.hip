// Persistent batched solver, instantiated for finest orders n0 = 2..5.
#include "batch.h"

namespace gllmg {

template <int N0>
void launch_batch_n(const BatchArgs& a, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_batch<N0>, dim3((unsigned)count), dim3(kBatchThreads), 0, s, a);
  GLLMG_HIP(hipGetLastError());
}

template void launch_batch_n<2>(const BatchArgs&, int, hipStream_t);
template void launch_batch_n<3>(const BatchArgs&, int, hipStream_t);
template void launch_batch_n<4>(const BatchArgs&, int, hipStream_t);
template void launch_batch_n<5>(const BatchArgs&, int, hipStream_t);

void launch_batch(int n0, const BatchArgs& a, int count, hipStream_t s) {
  switch (n0) {
#define GLLMG_CASE(NV) \
  case NV:             \
    return launch_batch_n<NV>(a, count, s);
    GLLMG_CASE(2) GLLMG_CASE(3) GLLMG_CASE(4) GLLMG_CASE(5) GLLMG_CASE(6) GLLMG_CASE(7)
    GLLMG_CASE(8) GLLMG_CASE(9) GLLMG_CASE(10) GLLMG_CASE(11) GLLMG_CASE(12) GLLMG_CASE(13)
    GLLMG_CASE(14) GLLMG_CASE(15) GLLMG_CASE(16) GLLMG_CASE(17)
#undef GLLMG_CASE
    default:
      throw Error(GLLMG_EINVAL, "unsupported order");
  }
}

}  // namespace gllmg
