// The work-queue batch kernels for complex<double> plans (queue_impl.h).
#include "queue_impl.h"

namespace nfft3 {
int launch_queue_f64(const QueueLaunch &q, hipStream_t s) { return launch_queue_t<double>(q, s); }
}  // namespace nfft3
