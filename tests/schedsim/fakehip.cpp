// Host-only stand-in for the HIP runtime calls of the library's host runtime
// (see fake/hip/hip_runtime.h).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <set>
#include <thread>

struct FakeStream {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::function<void()>> q;
    bool busy = false, stop = false;
    std::thread th;
    FakeStream()
    {
        th = std::thread([this] {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                cv.wait(lk, [&] { return stop || !q.empty(); });
                if (q.empty() && stop)
                    return;
                std::function<void()> fn = std::move(q.front());
                q.pop_front();
                busy = true;
                lk.unlock();
                fn();
                lk.lock();
                busy = false;
                cv.notify_all();
            }
        });
    }
    void push(std::function<void()> fn)
    {
        std::lock_guard<std::mutex> g(mu);
        q.push_back(std::move(fn));
        cv.notify_all();
    }
    void drain()
    {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return q.empty() && !busy; });
    }
    ~FakeStream()
    {
        {
            std::lock_guard<std::mutex> g(mu);
            stop = true;
            cv.notify_all();
        }
        th.join();
    }
};

struct FakeEvent {
    std::mutex mu;
    bool done = true;
    unsigned long long seq = 0;  // the latest record; an earlier one no longer counts
    double t = 0.0;              // seconds, when it completed
};

namespace {
std::mutex g_mu;
std::set<FakeStream *> g_streams;

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// the device-wide synchronisation of hipFree and hipHostFree
void sync_all()
{
    std::set<FakeStream *> all;
    {
        std::lock_guard<std::mutex> g(g_mu);
        all = g_streams;
    }
    for (FakeStream *s : all)
        s->drain();
}
}  // namespace

void fake_enqueue(hipStream_t s, std::function<void()> fn)
{
    if (s)
        s->push(std::move(fn));
    else
        fn();
}

hipError_t hipGetDeviceCount(int *count)
{
    *count = 1;
    return hipSuccess;
}
hipError_t hipSetDevice(int device) { return device == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t *prop, int)
{
    prop->multiProcessorCount = 256;
    std::strcpy(prop->gcnArchName, "fake");
    return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t bytes)
{
    *p = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p)
{
    sync_all();
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned) { return hipMalloc(p, bytes); }
hipError_t hipHostFree(void *p) { return hipFree(p); }
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind)
{
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t s)
{
    fake_enqueue(s, [=] { std::memcpy(dst, src, bytes); });
    return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind, hipStream_t s)
{
    fake_enqueue(s, [=] {
        for (size_t r = 0; r < height; r++)
            std::memcpy((char *)dst + r * dpitch, (const char *)src + r * spitch, width);
    });
    return hipSuccess;
}
hipError_t hipMemcpy2D(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                       hipMemcpyKind kind)
{
    return hipMemcpy2DAsync(dst, dpitch, src, spitch, width, height, kind, nullptr);
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    *s = new FakeStream();
    std::lock_guard<std::mutex> g(g_mu);
    g_streams.insert(*s);
    return hipSuccess;
}
hipError_t hipExtStreamCreateWithCUMask(hipStream_t *s, uint32_t words, const uint32_t *mask)
{
    if (!words || !mask)
        return hipErrorInvalidValue;
    return hipStreamCreateWithFlags(s, 0);
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_streams.erase(s);
    }
    s->drain();
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s)
{
    if (s)
        s->drain();
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = new FakeEvent();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    unsigned long long mine;
    {
        std::lock_guard<std::mutex> g(e->mu);
        e->done = false;
        mine = ++e->seq;
    }
    fake_enqueue(s, [e, mine] {
        std::lock_guard<std::mutex> g(e->mu);
        if (e->seq == mine) {
            e->done = true;
            e->t = now_s();
        }
    });
    return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e)
{
    std::lock_guard<std::mutex> g(e->mu);
    return e->done ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    std::lock_guard<std::mutex> ga(a->mu);
    std::lock_guard<std::mutex> gb(b->mu);
    if (!a->done || !b->done)
        return hipErrorNotReady;
    *ms = (float)(1e3 * (b->t - a->t));
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **p, const void *symbol)
{
    *p = (void *)symbol;
    return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
