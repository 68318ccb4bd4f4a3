// Host-only stand-in for the HIP runtime header, for the request loop's CPU
// self-tests (tests/host/serve_selftest.cpp, tests/host/split_selftest.cpp):
// events complete after a few queries, copies are memcpy, allocations are
// calloc. Nothing here runs on a GPU; the library itself is never built
// against it.
#pragma once
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#define __host__
#define __device__
#define __global__
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorNotReady = 600 };
typedef struct ihipStream_t *hipStream_t;
struct MockEvent {
    int polls_left;
    bool reported;   // completion already seen by a query
};
typedef MockEvent *hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
#define hipEventDisableTiming 2
#define hipHostMallocDefault 0
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned)
{
    *e = new MockEvent{0, true};
    return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t)
{
    e->polls_left = 2;
    e->reported = false;
    return hipSuccess;
}
// called when a query first sees a recorded event complete (a test's hook)
inline void (*mock_on_event_done)() = nullptr;
inline hipError_t hipEventQuery(hipEvent_t e)
{
    if (e->polls_left > 0) {
        e->polls_left--;
        return hipErrorNotReady;
    }
    if (!e->reported) {
        e->reported = true;
        if (mock_on_event_done)
            mock_on_event_done();
    }
    return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t e)
{
    e->polls_left = 0;
    return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t)
{
    std::memcpy(d, s, n);
    return hipSuccess;
}
template <class T>
hipError_t hipMalloc(T **p, size_t n)
{
    *p = (T *)std::calloc(1, n);
    return *p ? hipSuccess : 2;
}
template <class T>
hipError_t hipHostMalloc(T **p, size_t n, unsigned)
{
    *p = (T *)std::calloc(1, n);
    return *p ? hipSuccess : 2;
}
inline hipError_t hipFree(void *p)
{
    std::free(p);
    return hipSuccess;
}
inline hipError_t hipHostFree(void *p)
{
    std::free(p);
    return hipSuccess;
}
