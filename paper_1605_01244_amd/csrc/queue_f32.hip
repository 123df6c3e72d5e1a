// The work-queue batch kernels for complex<float> plans (queue_impl.h).
#include "queue_impl.h"

namespace nfft3 {
int launch_queue_f32(const QueueLaunch &q, hipStream_t s) { return launch_queue_t<float>(q, s); }
}  // namespace nfft3
