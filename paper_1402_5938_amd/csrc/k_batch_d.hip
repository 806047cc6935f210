// Persistent batched solver, instantiated for finest orders n0 = 14..17.
#include "batch.h"

namespace gllmg {

template <int N0>
void launch_batch_n(const BatchArgs& a, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_batch<N0>, dim3((unsigned)count), dim3(kBatchThreads), 0, s, a);
  GLLMG_HIP(hipGetLastError());
}

template void launch_batch_n<14>(const BatchArgs&, int, hipStream_t);
template void launch_batch_n<15>(const BatchArgs&, int, hipStream_t);
template void launch_batch_n<16>(const BatchArgs&, int, hipStream_t);
template void launch_batch_n<17>(const BatchArgs&, int, hipStream_t);

}  // namespace gllmg
