// Error reporting, pointer checks and allocation for the nsasm C ABI.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <atomic>

#include "internal.hpp"

namespace nsasm {

namespace {
thread_local std::string g_message;
thread_local KernelEvents g_kernel_events;
std::atomic<long> g_alloc_count{0};

long fail_alloc_at() {
    static const long k = [] {
        const char *s = std::getenv("NSASM_TEST_FAIL_ALLOC");
        return s ? std::atol(s) : 0L;
    }();
    return k;
}
}  // namespace

nsasm_status fail(nsasm_status status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_message = buf;
    return status;
}

void clear_error() { g_message.clear(); }

KernelEvents take_kernel_events() {
    KernelEvents e = g_kernel_events;
    g_kernel_events = KernelEvents{};
    return e;
}

nsasm_status hip_fail(hipError_t err, const char *what) {
    nsasm_status s = (err == hipErrorOutOfMemory || err == hipErrorMemoryAllocation)
                         ? NSASM_ERR_OUT_OF_MEMORY
                         : NSASM_ERR_DEVICE;
    return fail(s, "%s failed: %s (%d)", what, hipGetErrorString(err), static_cast<int>(err));
}

nsasm_status check_device_ptr(const void *p, const char *name) {
    if (p == nullptr) return fail(NSASM_ERR_INVALID_ARGUMENT, "%s is NULL", name);
    hipPointerAttribute_t attr{};
    hipError_t err = hipPointerGetAttributes(&attr, p);
    if (err != hipSuccess) {
        (void)hipGetLastError();  // do not leave the error for the next call
        return fail(NSASM_ERR_INVALID_ARGUMENT, "%s is not a device pointer (%s)", name,
                    hipGetErrorString(err));
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(NSASM_ERR_INVALID_ARGUMENT, "%s is not device memory (memory type %d)", name,
                    static_cast<int>(attr.type));
    return NSASM_OK;
}

nsasm_status device_alloc(void **p, size_t bytes, const char *what) {
    *p = nullptr;
    long k = ++g_alloc_count;
    if (fail_alloc_at() > 0 && k == fail_alloc_at())
        return fail(NSASM_ERR_OUT_OF_MEMORY, "allocation of %zu bytes for %s failed (injected)",
                    bytes, what);
    if (bytes == 0) bytes = 1;
    hipError_t err = hipMalloc(p, bytes);
    if (err != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(NSASM_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes for %s failed: %s", bytes,
                    what, hipGetErrorString(err));
    }
    return NSASM_OK;
}

void device_free(void *p) {
    if (p) (void)hipFree(p);
}

}  // namespace nsasm

extern "C" const char *nsasm_last_error(void) { return nsasm::g_message.c_str(); }

extern "C" nsasm_status nsasm_set_kernel_events(void *element_start, void *element_stop, void *gather_start,
                                                void *gather_stop) {
    nsasm::g_kernel_events = nsasm::KernelEvents{
        static_cast<hipEvent_t>(element_start), static_cast<hipEvent_t>(element_stop),
        static_cast<hipEvent_t>(gather_start), static_cast<hipEvent_t>(gather_stop)};
    nsasm::clear_error();
    return NSASM_OK;
}

extern "C" const char *nsasm_version(void) { return "0.2.0"; }
