// Host stand-in for the few HIP runtime calls the library's scheduling and
// serving code makes (test infrastructure: lets the serving loop and the
// batch scheduler run on a machine without a GPU, under the address and
// undefined-behaviour sanitizers).
//
// "Device" memory is host memory, and every enqueued operation runs at
// once on the calling thread, so a stream is always drained and an event
// always complete.  Allocations are tracked: freeing an unknown pointer
// aborts, and fake_hip_set_capacity() caps the live device bytes so that
// out-of-memory paths can be exercised.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>

namespace {

struct State {
    std::mutex mu;
    std::map<void*, size_t> dev, host;
    std::set<void*> streams, events;
    size_t live = 0, peak = 0, cap = (size_t)1 << 40;
};
State& st() {
    static State* s = new State;
    return *s;
}

[[noreturn]] void die(const char* what, const void* p) {
    std::fprintf(stderr, "fake_hip: %s %p\n", what, p);
    std::abort();
}

void* aligned(size_t bytes) {
    const size_t b = (bytes + 255) / 256 * 256;
    void* p = std::aligned_alloc(256, b ? b : 256);
    if (p) std::memset(p, 0xA5, b ? b : 256);   // device memory starts undefined
    return p;
}

}  // namespace

extern "C" {

void fake_hip_set_capacity(size_t bytes) {
    std::lock_guard<std::mutex> g(st().mu);
    st().cap = bytes;
}
size_t fake_hip_live_bytes() {
    std::lock_guard<std::mutex> g(st().mu);
    return st().live;
}
size_t fake_hip_peak_bytes() {
    std::lock_guard<std::mutex> g(st().mu);
    return st().peak;
}
int fake_hip_live_objects() {
    std::lock_guard<std::mutex> g(st().mu);
    return (int)(st().dev.size() + st().host.size() + st().streams.size() + st().events.size());
}

const char* hipGetErrorString(hipError_t e) {
    return e == hipErrorOutOfMemory ? "out of memory (fake)" : "device error (fake)";
}

hipError_t hipSetDevice(int) { return hipSuccess; }

hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int) {
    std::memset(prop, 0, sizeof(*prop));
    std::strcpy(prop->gcnArchName, "fake-host");
    return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }

hipError_t hipMalloc(void** p, size_t bytes) {
    State& s = st();
    std::lock_guard<std::mutex> g(s.mu);
    if (s.live + bytes > s.cap) return hipErrorOutOfMemory;
    *p = aligned(bytes);
    if (!*p) return hipErrorOutOfMemory;
    s.dev[*p] = bytes;
    s.live += bytes;
    if (s.live > s.peak) s.peak = s.live;
    return hipSuccess;
}

hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    State& s = st();
    std::lock_guard<std::mutex> g(s.mu);
    auto it = s.dev.find(p);
    if (it == s.dev.end()) die("hipFree of an unknown pointer", p);
    s.live -= it->second;
    s.dev.erase(it);
    std::free(p);
    return hipSuccess;
}

hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) {
    State& s = st();
    std::lock_guard<std::mutex> g(s.mu);
    *p = aligned(bytes);
    if (!*p) return hipErrorOutOfMemory;
    s.host[*p] = bytes;
    return hipSuccess;
}

hipError_t hipHostFree(void* p) {
    if (!p) return hipSuccess;
    State& s = st();
    std::lock_guard<std::mutex> g(s.mu);
    auto it = s.host.find(p);
    if (it == s.host.end()) die("hipHostFree of an unknown pointer", p);
    s.host.erase(it);
    std::free(p);
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* out, unsigned int) {
    void* h = std::malloc(1);
    std::lock_guard<std::mutex> g(st().mu);
    st().streams.insert(h);
    *out = reinterpret_cast<hipStream_t>(h);
    return hipSuccess;
}

hipError_t hipStreamDestroy(hipStream_t s) {
    std::lock_guard<std::mutex> g(st().mu);
    if (!st().streams.erase(s)) die("hipStreamDestroy of an unknown stream", s);
    std::free(s);
    return hipSuccess;
}

static void check_stream(hipStream_t s) {
    if (!s) return;   // the null stream
    std::lock_guard<std::mutex> g(st().mu);
    if (!st().streams.count(s)) die("use of an unknown stream", s);
}

static void check_event(hipEvent_t e) {
    std::lock_guard<std::mutex> g(st().mu);
    if (!st().events.count(e)) die("use of an unknown event", e);
}

hipError_t hipStreamSynchronize(hipStream_t s) {
    check_stream(s);
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* out, unsigned int) {
    void* h = std::malloc(1);
    std::lock_guard<std::mutex> g(st().mu);
    st().events.insert(h);
    *out = reinterpret_cast<hipEvent_t>(h);
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* out) { return hipEventCreateWithFlags(out, 0); }

hipError_t hipEventDestroy(hipEvent_t e) {
    std::lock_guard<std::mutex> g(st().mu);
    if (!st().events.erase(e)) die("hipEventDestroy of an unknown event", e);
    std::free(e);
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    check_event(e);
    check_stream(s);
    return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t e) {
    check_event(e);
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e) {
    check_event(e);
    return hipSuccess;
}

hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    check_event(a);
    check_event(b);
    *ms = 0.0f;
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
    check_stream(s);
    check_event(e);
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
    check_stream(s);
    if (bytes) std::memcpy(dst, src, bytes);
    return hipSuccess;
}

hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                            size_t height, hipMemcpyKind, hipStream_t s) {
    check_stream(s);
    for (size_t r = 0; r < height; ++r)
        std::memcpy(static_cast<char*>(dst) + r * dpitch, static_cast<const char*>(src) + r * spitch, width);
    return hipSuccess;
}

hipError_t hipMemsetAsync(void* dst, int v, size_t bytes, hipStream_t s) {
    check_stream(s);
    std::memset(dst, v, bytes);
    return hipSuccess;
}

}  // extern "C"
