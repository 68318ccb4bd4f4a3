// Store-only probe: the write ceiling of an output layout.
//
// A measurement aid beside the generator library, with no generator code in
// it. Wavefronts pop output ranges from a queue (one range per wavefront at a
// time, as the generation kernels take their work items) and fill each range
// front to back, 64 lanes x `width` consecutive words per store instruction,
// eight such stores per buffer window. With width 1 that is the generation
// kernels' own store pattern (one 4-byte word per lane, 256 bytes per
// instruction); widths 2 and 4 show what wider stores would gain. The time of
// such a launch bounds from below what any kernel writing the same ranges in
// the same order can reach.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace {

struct ProbeItem {
    uint64_t out;   // device address of the range (4-byte aligned)
    uint64_t n;     // words in the range
};

typedef uint32_t u2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

constexpr int kWord3 = 0x00020000;   // gfx9-family buffer descriptor word 3 (32-bit data format)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t window(uint64_t addr, uint32_t words)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)addr);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32));
    uint32_t *p = reinterpret_cast<uint32_t *>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(static_cast<void *>(p), 0,
                                             (int)__builtin_amdgcn_readfirstlane(words * 4u), kWord3);
}

template <int WIDTH, int POLICY>
__device__ __forceinline__ void put(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t v)
{
    if constexpr (WIDTH == 1)
        __builtin_amdgcn_raw_buffer_store_b32(v, rs, (int)off, 0, POLICY);
    else if constexpr (WIDTH == 2)
        __builtin_amdgcn_raw_buffer_store_b64(u2v{v, v ^ 1u}, rs, (int)off, 0, POLICY);
    else
        __builtin_amdgcn_raw_buffer_store_b128(u4v{v, v ^ 1u, v ^ 2u, v ^ 3u}, rs, (int)off, 0, POLICY);
}

// counter[0]: queue head; counter[1]: wavefronts done (the last one resets
// both, so the next launch starts from zero)
template <int WIDTH, int POLICY>
__global__ __launch_bounds__(64) void store_probe_kernel(const ProbeItem *__restrict__ items, uint32_t nitems,
                                                         uint32_t *counter)
{
    const uint32_t lane = threadIdx.x;
    constexpr uint32_t CH = 64u * WIDTH;   // words per store instruction
    for (;;) {
        uint32_t q = 0;
        if (lane == 0)
            q = atomicAdd(&counter[0], 1u);
        q = __builtin_amdgcn_readfirstlane(q);
        if (q >= nitems)
            break;
        const uint64_t out = items[q].out, n = items[q].n;
        uint64_t k = 0;
        for (; k < n; k += 8 * CH) {
            const uint64_t left = n - k;
            const __amdgpu_buffer_rsrc_t rs = window(out + 4 * k, (uint32_t)(left < 8 * CH ? left : 8 * CH));
#pragma unroll
            for (uint32_t j = 0; j < 8; j++)
                put<WIDTH, POLICY>(rs, 4u * (j * CH + lane * WIDTH), q + j + lane);
        }
    }
    if (lane == 0) {
        const uint32_t done = atomicAdd(&counter[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&counter[0], 0u);
            atomicExch(&counter[1], 0u);
        }
    }
}

__global__ void zero2(uint32_t *c)
{
    if (threadIdx.x < 2)
        c[threadIdx.x] = 0;
}

template <int WIDTH, int POLICY>
hipError_t launch(const ProbeItem *d, uint32_t nitems, uint32_t *counter, uint32_t waves, hipStream_t s)
{
    hipLaunchKernelGGL((store_probe_kernel<WIDTH, POLICY>), dim3(waves), dim3(64), 0, s, d, nitems, counter);
    return hipGetLastError();
}

}  // namespace

extern "C" {

// Average time in ms of `reps` store-only launches of `waves` wavefronts
// (one per 64-lane workgroup) filling the ranges outs[i] .. outs[i] + 4 ns[i]
// bytes, popped in the given order; width 1, 2 or 4 words per lane and
// store; nontemporal 0 (plain stores) or 1. Returns 0, or -1 for bad
// arguments (no ranges, a range not 4-byte aligned or with n = 0, width not
// 1/2/4, waves 0, reps 0), -3 on a HIP error.
int mtgp_probe_store_ms(const uint64_t *outs, const uint64_t *ns, uint32_t nitems, uint32_t waves, uint32_t width,
                        int nontemporal, uint32_t reps, void *stream, float *ms)
{
    if (!outs || !ns || !ms || nitems == 0 || waves == 0 || reps == 0 || (width != 1 && width != 2 && width != 4))
        return -1;
    std::vector<ProbeItem> h(nitems);
    for (uint32_t i = 0; i < nitems; i++) {
        if ((outs[i] & 3u) != 0 || ns[i] == 0)
            return -1;
        h[i] = ProbeItem{outs[i], ns[i]};
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    ProbeItem *d = nullptr;
    uint32_t *counter = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    auto run = [&]() -> hipError_t {
        const int sel = (int)width * 2 + (nontemporal ? 1 : 0);
        switch (sel) {
        case 2: return launch<1, 0>(d, nitems, counter, waves, s);
        case 3: return launch<1, 2>(d, nitems, counter, waves, s);
        case 4: return launch<2, 0>(d, nitems, counter, waves, s);
        case 5: return launch<2, 2>(d, nitems, counter, waves, s);
        case 8: return launch<4, 0>(d, nitems, counter, waves, s);
        default: return launch<4, 2>(d, nitems, counter, waves, s);
        }
    };
    if (hipMalloc(&d, nitems * sizeof(ProbeItem)) != hipSuccess || hipMalloc(&counter, 2 * sizeof(uint32_t)) != hipSuccess ||
        hipMemcpyAsync(d, h.data(), nitems * sizeof(ProbeItem), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = -3;
    } else {
        hipLaunchKernelGGL(zero2, dim3(1), dim3(64), 0, s, counter);
        bool ok = hipGetLastError() == hipSuccess && run() == hipSuccess;   // warm-up
        float total = 0.0f;
        for (uint32_t r = 0; ok && r < reps; r++) {
            float t = 0.0f;
            ok = hipEventRecord(e0, s) == hipSuccess && run() == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
            total += t;
        }
        if (ok)
            *ms = total / (float)reps;
        else
            rc = -3;
    }
    if (hipStreamSynchronize(s) != hipSuccess)
        rc = -3;
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(d);
    (void)hipFree(counter);
    return rc;
}

}  // extern "C"
