// Per-kernel timing with HIP events (jas_timing_enable / jas_timing_report).
#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "jas_internal.hpp"

namespace jas {
namespace {

struct Pending {
    const char *name;
    hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::map<std::string, std::pair<uint64_t, double>> g_acc;
std::vector<std::string> g_names;  // stable storage for reported names

}  // namespace

bool timing_on() { return g_on; }

KernelTimer::KernelTimer(const char *name, hipStream_t s) : name_(name), s_(s) {
    if (!g_on) return;
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) {
        (void)hipGetLastError();
        a_ = b_ = nullptr;
        return;
    }
    (void)hipEventRecord(a_, s_);
}

KernelTimer::~KernelTimer() {
    if (!a_) return;
    (void)hipEventRecord(b_, s_);
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back({name_, a_, b_});
}

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

HostTimer::HostTimer(const char *name) : name_(name) {
    if (g_on) t0_ = now_ms();
}

HostTimer::~HostTimer() {
    if (t0_ < 0) return;
    const double dt = now_ms() - t0_;
    std::lock_guard<std::mutex> lk(g_mu);
    auto &e = g_acc[std::string("host:") + name_];
    e.first += 1;
    e.second += dt;
}

}  // namespace jas

extern "C" {

void jas_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(jas::g_mu);
    jas::g_on = on != 0;
}

int32_t jas_timing_report(jas_kernel_time *out, int32_t cap) {
    std::lock_guard<std::mutex> lk(jas::g_mu);
    for (auto &p : jas::g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto &e = jas::g_acc[p.name];
            e.first += 1;
            e.second += ms;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    (void)hipGetLastError();
    jas::g_pending.clear();
    std::vector<std::pair<std::string, std::pair<uint64_t, double>>> v(jas::g_acc.begin(), jas::g_acc.end());
    std::sort(v.begin(), v.end(), [](const auto &x, const auto &y) { return x.second.second > y.second.second; });
    const int32_t count = (int32_t)v.size();
    jas::g_names.clear();
    for (auto &e : v) jas::g_names.push_back(e.first);
    for (int32_t k = 0; k < count && k < cap && out; ++k) {
        out[k].name = jas::g_names[k].c_str();
        out[k].launches = v[k].second.first;
        out[k].total_ms = v[k].second.second;
    }
    jas::g_acc.clear();
    return count;
}

}  // extern "C"
