// lra_probe.hip -- measurement helper: the latency of one exchange between
// workgroups on different XCDs, the unit of the team selections' critical
// path (each selection waits for at least one such hop).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lra_internal.h"

namespace lra {
namespace {

// Two workgroups of one cooperative launch (consecutive workgroups are dealt
// to different XCDs) pass a counter back and forth through one 64-bit word
// with device-scope relaxed atomics, the accesses of the team exchange.  Round
// k: workgroup k mod 2 stores k + 1, the other polls until it reads k + 1.
// Every poll is bounded in wall-clock time (`limit` ticks); past it the
// workgroup stops and flags the failure, so the launch always ends.
// out[0] = ticks from the first store to the last read (workgroup 0),
// out[1] = rounds completed, out[2] = 1 on a timeout.
__global__ void __launch_bounds__(64) xlat_kernel(uint64_t *word, int rounds, uint64_t limit, uint64_t *out) {
    if (threadIdx.x != 0) return;
    const int me = (int)blockIdx.x;
    const uint64_t t0 = wall_clock64();
    int k = 0;
    bool fail = false;
    for (; k < rounds && !fail; k++) {
        if ((k & 1) == me) {
            __hip_atomic_store(word, (uint64_t)(k + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t w0 = wall_clock64();
            while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != (uint64_t)(k + 1)) {
                if (wall_clock64() - w0 > limit) {
                    fail = true;
                    break;
                }
            }
        }
    }
    if (me == 0) {
        out[0] = wall_clock64() - t0;
        out[1] = (uint64_t)k;
    }
    if (fail) out[2] = 1;
}

__global__ void xlat_clear_kernel(uint64_t *p) {
    if (threadIdx.x < 4) p[threadIdx.x] = 0;
}

}  // namespace

hipError_t launch_xlat(uint64_t *buf, int rounds, uint64_t limit, hipStream_t stream) {
    hipLaunchKernelGGL(xlat_clear_kernel, dim3(1), dim3(64), 0, stream, buf);
    uint64_t *word = buf + 3, *out = buf;
    void *args[] = {(void *)&word, (void *)&rounds, (void *)&limit, (void *)&out};
    return hipLaunchCooperativeKernel((const void *)xlat_kernel, dim3(2), dim3(64), args, 0, stream);
}

}  // namespace lra
