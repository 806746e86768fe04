// api.hip -- error reporting, launch configuration, device queries, utility
// kernels and the HIP graph helpers of libfem.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "fem_internal.h"

namespace fem {

namespace {
thread_local char g_err[512] = "";

std::mutex g_cfg_mu;
bool g_cfg_set[2][2] = {{false, false}, {false, false}};
fem_launch g_cfg[2][2];

int g_cu_count[64] = {0};

std::atomic<int> g_timing{0};
struct TimedLaunch {
    int kernel;
    hipEvent_t start, stop;
};
std::mutex g_time_mu;
std::vector<TimedLaunch> g_launches;
}  // namespace

bool timing_on() { return g_timing.load(std::memory_order_relaxed) != 0; }

void* timing_begin(hipStream_t s) {
    if (!timing_on()) return nullptr;
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    if (hipEventRecord(ev, s) != hipSuccess) {
        (void)hipEventDestroy(ev);
        return nullptr;
    }
    return (void*)ev;
}

void timing_end(void* token, int kernel, hipStream_t s) {
    if (!token) return;
    hipEvent_t stop = nullptr;
    if (hipEventCreate(&stop) != hipSuccess || hipEventRecord(stop, s) != hipSuccess) {
        (void)hipEventDestroy((hipEvent_t)token);
        if (stop) (void)hipEventDestroy(stop);
        return;
    }
    std::lock_guard<std::mutex> lk(g_time_mu);
    g_launches.push_back(TimedLaunch{kernel, (hipEvent_t)token, stop});
}

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

int device_cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev < 0 || dev >= 64) return 256;
    if (g_cu_count[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        g_cu_count[dev] = n;
    }
    return g_cu_count[dev];
}

static fem_launch default_launch(int kernel, int prec) {
    // measured on MI355X (100^3 cube, 200x200x2 voided specimen): both element
    // kernels are fastest with one wave per workgroup in both precisions
    fem_launch c;
    c.block = 64;
    c.waves_per_cu = 8;
    c.xcd_remap = 1;
    (void)kernel;
    (void)prec;
    return c;
}

fem_launch launch_config(int kernel, int prec) {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    if (kernel >= 0 && kernel < 2 && prec >= 0 && prec < 2 && g_cfg_set[kernel][prec])
        return g_cfg[kernel][prec];
    return default_launch(kernel, prec);
}

int persistent_grid(const fem_launch& cfg, int64_t n_tiles) {
    int64_t blocks = (int64_t)cfg.waves_per_cu * device_cu_count() * 64 / cfg.block;
    if (blocks < 8) blocks = 8;
    blocks = (blocks + 7) / 8 * 8;  // a multiple of the XCD count
    if (blocks > n_tiles) blocks = n_tiles;
    if (blocks < 1) blocks = 1;
    return (int)blocks;
}

__global__ void zero_kernel(uint4* p16, size_t n16, unsigned char* tail, size_t ntail) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (; i < n16; i += stride) p16[i] = z;
    if (blockIdx.x == 0)
        for (size_t t = threadIdx.x; t < ntail; t += blockDim.x) tail[t] = 0;
}

__global__ void zero_counters_kernel(int32_t* a, int na, int32_t* b, int nb) {
    const int t = (int)threadIdx.x;
    if (a && t < na) a[t] = 0;
    if (b && t < nb) b[t] = 0;
}

hipError_t zero_counters(int32_t* a, int na, int32_t* b, int nb, hipStream_t s) {
    if ((!a || na <= 0) && (!b || nb <= 0)) return hipSuccess;
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, s, a, na, b, nb);
    return hipGetLastError();
}

hipError_t zero_bytes(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0 || p == nullptr) return hipSuccess;
    // leading bytes up to 16-byte alignment go to the tail path
    uintptr_t a = reinterpret_cast<uintptr_t>(p);
    size_t lead = (16 - (a & 15)) & 15;
    if (lead > bytes) lead = bytes;
    unsigned char* c = static_cast<unsigned char*>(p);
    if (lead) hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, nullptr, (size_t)0, c, lead);
    size_t rest = bytes - lead;
    size_t n16 = rest / 16, ntail = rest % 16;
    int threads = 256;
    size_t blocks = (n16 + threads - 1) / threads;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(threads), 0, s,
                       reinterpret_cast<uint4*>(c + lead), n16, c + lead + n16 * 16, ntail);
    return hipGetLastError();
}

}  // namespace fem

using namespace fem;

extern "C" {

int fem_version(void) { return 100; }

const char* fem_last_error(void) { return g_err; }

int fem_set_launch(int kernel, fem_precision prec, const fem_launch* cfg) {
    if (prec == FEM_FP64_K32) prec = FEM_FP64;  // the same element kernels as FEM_FP64
    if (kernel < 0 || kernel > 1 || (int)prec < 0 || (int)prec > 1)
        return set_error(FEM_EINVAL, "fem_set_launch: bad kernel %d or precision %d", kernel, (int)prec);
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    if (!cfg) {
        g_cfg_set[kernel][prec] = false;
        return FEM_OK;
    }
    if (!(cfg->block == 64 || cfg->block == 128 || cfg->block == 256) || cfg->waves_per_cu < 1 ||
        cfg->waves_per_cu > 64)
        return set_error(FEM_EINVAL, "fem_set_launch: block must be 64/128/256 and waves_per_cu in [1,64]");
    g_cfg[kernel][prec] = *cfg;
    g_cfg_set[kernel][prec] = true;
    return FEM_OK;
}

int fem_get_launch(int kernel, fem_precision prec, fem_launch* cfg) {
    if (prec == FEM_FP64_K32) prec = FEM_FP64;
    if (!cfg || kernel < 0 || kernel > 1 || (int)prec < 0 || (int)prec > 1)
        return set_error(FEM_EINVAL, "fem_get_launch: bad arguments");
    *cfg = launch_config(kernel, prec);
    return FEM_OK;
}

int fem_timing_enable(int on) {
    g_timing.store(on ? 1 : 0);
    return FEM_OK;
}

int fem_timing_read(int kernel, double* total_ms, int32_t* launches) {
    if (!total_ms || !launches) return set_error(FEM_EINVAL, "fem_timing_read: NULL output");
    std::vector<TimedLaunch> keep, mine;
    {
        std::lock_guard<std::mutex> lk(g_time_mu);
        for (auto& t : g_launches) (t.kernel == kernel ? mine : keep).push_back(t);
        g_launches.swap(keep);
    }
    double sum = 0.0;
    int err = 0;
    for (auto& t : mine) {
        float ms = 0.f;
        if (hipEventSynchronize(t.stop) != hipSuccess || hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess)
            err = 1;
        sum += ms;
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    *total_ms = sum;
    *launches = (int32_t)mine.size();
    return err ? set_error(FEM_EHIP, "fem_timing_read: event query failed") : FEM_OK;
}

int fem_graph_begin(void* stream) {
    FEM_HIP_CHECK(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return FEM_OK;
}

int fem_graph_end(void* stream, void** graph_exec) {
    if (!graph_exec) return set_error(FEM_EINVAL, "fem_graph_end: graph_exec is NULL");
    hipGraph_t g = nullptr;
    FEM_HIP_CHECK(hipStreamEndCapture((hipStream_t)stream, &g));
    hipGraphExec_t ex = nullptr;
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess)
        return set_error(FEM_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    *graph_exec = (void*)ex;
    return FEM_OK;
}

int fem_graph_launch(void* graph_exec, void* stream) {
    if (!graph_exec) return set_error(FEM_EINVAL, "fem_graph_launch: graph_exec is NULL");
    FEM_HIP_CHECK(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream));
    return FEM_OK;
}

int fem_graph_destroy(void* graph_exec) {
    if (!graph_exec) return FEM_OK;
    FEM_HIP_CHECK(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
    return FEM_OK;
}

}  // extern "C"
