// prof.hip -- stage timing for the benchmark: when enabled, every stage launch is bracketed by
// two HIP events recorded on the stream it is launched on; digs_profile_read synchronises,
// converts the event pairs to durations and sums them per stage. Not thread-safe; meant for a
// single benchmarking thread. Events are pooled and reused across reads.
#include <string.h>

#include <vector>

#include "prof.h"

static bool g_on = false;

struct Pending {
    int stage;
    hipEvent_t a, b;
};

static std::vector<Pending> g_pending;
static std::vector<hipEvent_t> g_pool;
static Pending g_open[PS_COUNT];
static double g_total_ms[PS_COUNT];
static long g_launches[PS_COUNT];

static const char *kNames[PS_COUNT] = {"ffd_canonical", "setup",     "scan",
                                       "bin_count",     "bin_fill",  "splat_fwd",
                                       "splat_bwd",     "cell_sort", "gauss_bwd",
                                       "coef_grad",     "other"};

static hipEvent_t take_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static thread_local int t_suppress = 0;

bool prof_on() { return g_on && t_suppress == 0; }

ProfSuppress::ProfSuppress() { ++t_suppress; }
ProfSuppress::~ProfSuppress() { --t_suppress; }

void prof_begin(int stage, hipStream_t s)
{
    Pending p;
    p.stage = stage;
    p.a = take_event();
    p.b = nullptr;
    if (p.a) hipEventRecord(p.a, s);
    g_open[stage] = p;
}

void prof_end(int stage, hipStream_t s)
{
    Pending p = g_open[stage];
    if (!p.a) return;
    p.b = take_event();
    if (!p.b) return;
    hipEventRecord(p.b, s);
    g_pending.push_back(p);
    g_open[stage].a = nullptr;
}

extern "C" int digs_profile_enable(int on)
{
    const int prev = g_on ? 1 : 0;
    if (on >= 0) g_on = on != 0;
    return prev;
}

extern "C" int digs_profile_read(digs_profile_entry *out, int max_entries, int reset)
{
    for (const Pending &p : g_pending) {
        if (hipEventSynchronize(p.b) != hipSuccess) return DIGS_EHIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_total_ms[p.stage] += ms;
            g_launches[p.stage] += 1;
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
    int k = 0;
    for (int s = 0; s < PS_COUNT && k < max_entries; ++s) {
        if (!out) break;
        strncpy(out[k].name, kNames[s], sizeof(out[k].name) - 1);
        out[k].name[sizeof(out[k].name) - 1] = 0;
        out[k].launches = g_launches[s];
        out[k].total_ms = g_total_ms[s];
        ++k;
    }
    if (reset) {
        memset(g_total_ms, 0, sizeof(g_total_ms));
        memset(g_launches, 0, sizeof(g_launches));
    }
    return k;
}
