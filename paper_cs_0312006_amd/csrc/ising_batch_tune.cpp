// Batch plan model and its autotuner.
//
// A batch of independent lattices (Section 2.2's sweeps, one Markov chain
// per lattice) runs either resident (each workgroup takes whole lattices
// and runs all their sweeps from its local memory) or stepped (every sweep
// is one launch over the tiles of all lattices). Which is faster, and which
// tile height the stepped walk should use, depends on the mix of sides and
// fields, so ISING_BATCH_AUTO predicts each plan's time from rates per
// lattice class:
//   resident: site updates per ns of one workgroup on one lattice of the
//     class, plus a fixed time per lattice (taking it from the queue and,
//     bit-packed, converting it to bits and back); the launch runs `slots`
//     workgroups and hands lattices out largest work first, so its time is
//     that queue's makespan;
//   stepped: site updates per ns of the whole GPU on lattices of the class,
//     for each tile height, scaled up when the batch has fewer tiles than
//     the GPU has wave slots, and never below one launch per sweep.
// A class is a side band (up to 128, 256, 512 and 1072, and larger: how the
// resident kernel holds a lattice, and how many tiles the stepped walk cuts
// it into) and whether the acceptance table needs the general bit-packed
// update (a field: one compare per (spin, m) class rather than two).
//
// ising_batch_tune measures these rates on the device with synthetic
// batches of each class (hot starts, J = 1, T spread over [1.5, 3.5],
// h = 0 or 0.05) and keeps them per device and, if asked, in a cache file
// keyed by the device's architecture and unit counts. Until a device is
// tuned the built-in rates, measured the same way on an MI355X, are used.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

#include "ising.h"
#include "ising_launch.hpp"
#include "ising_runtime.hpp"

using namespace ising;

namespace {

constexpr int kBands = 5;
constexpr int kClasses = 2 * kBands;
constexpr int kRowChoices = 3;
constexpr uint32_t kRows[kRowChoices] = {8, 16, 32};
// upper side of each band but the last, and the side a band's trials use
constexpr uint32_t kBandMax[kBands - 1] = {128, 256, 512, 1072};
constexpr uint32_t kBandSide[kBands] = {128, 256, 512, 1024, 2048};
constexpr double kTrialField = 0.05;

struct Rates {
    bool tuned = false;
    double res[kClasses];              // resident, per workgroup
    double res_fixed[kClasses];        // resident, ns per lattice
    double st[kClasses][kRowChoices];  // stepped, whole GPU
    double floor_ns;                   // stepped: least time per sweep
};

// Built-in rates (site updates per ns), from ising_batch_tune on an MI355X.
const Rates kDefaultRates = {
    false,
    // resident, per workgroup: bands 128, 256, 512, 1072, larger; h = 0 then h != 0
    {5.45, 4.05, 8.59, 6.08, 9.06, 6.05, 9.02, 6.31, 5.11, 5.12},
    // resident, fixed ns per lattice
    {72e3, 104e3, 147e3, 118e3, 169e3, 187e3, 381e3, 406e3, 20e3, 22e3},
    // stepped, tile rows 8, 16, 32
    {{323, 220, 138}, {318, 220, 137},
     {841, 758, 505}, {841, 756, 502},
     {1302, 1312, 1222}, {1282, 1296, 1209},
     {1476, 1710, 1668}, {1498, 1729, 1697},
     {1798, 1981, 2008}, {1799, 1984, 2004}},
    11792.0,
};

constexpr int kMaxDevices = 64;
std::mutex g_mu;
Rates g_rates[kMaxDevices];
bool g_have[kMaxDevices] = {false};

Rates rates_for(int dev) {
    std::lock_guard<std::mutex> g(g_mu);
    if (dev >= 0 && dev < kMaxDevices && g_have[dev]) return g_rates[dev];
    return kDefaultRates;
}

int band_of(uint32_t L) {
    for (int b = 0; b < kBands - 1; ++b)
        if (L <= kBandMax[b]) return b;
    return kBands - 1;
}

int class_of(uint32_t L, const AcceptTable& at) { return 2 * band_of(L) + (bits_mode(at) == 3u ? 1 : 0); }

// Largest workgroup load when the times are handed out largest first to
// the least loaded of `slots` workgroups (the resident queue's order).
double makespan(std::vector<double> t, uint32_t slots) {
    std::sort(t.begin(), t.end(), std::greater<double>());
    std::priority_queue<double, std::vector<double>, std::greater<double>> load;
    for (uint32_t k = 0; k < slots; ++k) load.push(0.0);
    double span = 0.0;
    for (double x : t) {
        const double l = load.top() + x;
        load.pop();
        load.push(l);
        span = std::max(span, l);
    }
    return span;
}

std::string device_key(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return std::string();
    }
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s cus=%d slots=%u fslots=%u", prop.gcnArchName, prop.multiProcessorCount,
                  engine_resident_slots(dev), engine_fused_slots(dev));
    for (char* c = buf; *c; ++c)
        if (*c == '\n') *c = ' ';
    return std::string(buf);
}

constexpr const char* kCacheMagic = "ising-batch-rates 2";

bool load_cache(const char* path, const std::string& key, Rates* out) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool ok = std::fgets(line, sizeof line, f) && std::strncmp(line, kCacheMagic, std::strlen(kCacheMagic)) == 0;
    if (ok) {
        line[std::strcspn(line, "\n")] = 0;
        ok = std::string(line + std::strlen(kCacheMagic)) == " " + key;
    }
    Rates r;
    int seen = 0;
    bool floor_seen = false;
    while (ok && std::fgets(line, sizeof line, f)) {
        int c = -1;
        double a, fx, b0, b1, b2;
        if (std::sscanf(line, "floor_ns %lf", &a) == 1) {
            ok = std::isfinite(a) && a > 0;
            r.floor_ns = a;
            floor_seen = true;
        } else if (std::sscanf(line, "class %d %lf %lf %lf %lf %lf", &c, &a, &fx, &b0, &b1, &b2) == 6) {
            ok = c >= 0 && c < kClasses && !(seen >> c & 1) && a > 0 && fx >= 0 && b0 > 0 && b1 > 0 && b2 > 0 &&
                 std::isfinite(a + fx + b0 + b1 + b2);
            if (ok) {
                r.res[c] = a;
                r.res_fixed[c] = fx;
                r.st[c][0] = b0;
                r.st[c][1] = b1;
                r.st[c][2] = b2;
                seen |= 1 << c;
            }
        } else {
            ok = false;
        }
    }
    std::fclose(f);
    if (!ok || !floor_seen || seen != (1 << kClasses) - 1) return false;
    r.tuned = true;
    *out = r;
    return true;
}

bool save_cache(const char* path, const std::string& key, const Rates& r) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "%s %s\n", kCacheMagic, key.c_str());
    std::fprintf(f, "floor_ns %.6g\n", r.floor_ns);
    for (int c = 0; c < kClasses; ++c)
        std::fprintf(f, "class %d %.6g %.6g %.6g %.6g %.6g\n", c, r.res[c], r.res_fixed[c], r.st[c][0], r.st[c][1],
                     r.st[c][2]);
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

struct TrialSet {
    std::vector<ising_ctx*> ctxs;
    ~TrialSet() {
        for (ising_ctx* c : ctxs) ising_destroy(c);
    }
};

// Time of `sweeps` sweeps of every lattice in the set (ns, best of two,
// after a warm-up that captures the plan's graphs).
int time_batch(TrialSet& set, uint64_t sweeps, bool stepped, uint32_t rows, hipStream_t s, hipEvent_t e0,
               hipEvent_t e1, double* ns) {
    const size_t count = set.ctxs.size();
    std::vector<uint64_t> warm(count, stepped ? 16u : 1u), n(count, sweeps);
    int rc = engine_run(set.ctxs.data(), warm.data(), count, s, stepped, rows);
    if (rc != ISING_OK) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return ISING_EDEVICE;
    double best = 0.0;
    for (int rep = 0; rep < 2; ++rep) {
        // the trials' series are not read: each run writes from the start of
        // the room reserved for it, so no run grows a series while timed
        for (ising_ctx* c : set.ctxs) c->series_len = 0;
        if (hipEventRecord(e0, s) != hipSuccess) return ISING_EDEVICE;
        rc = engine_run(set.ctxs.data(), n.data(), count, s, stepped, rows);
        if (rc != ISING_OK) return rc;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return ISING_EDEVICE;
        const double t = (double)ms * 1e6;
        if (rep == 0 || t < best) best = t;
    }
    for (ising_ctx* c : set.ctxs) c->series_len = 0;
    *ns = best;
    return ISING_OK;
}

int make_set(TrialSet& set, uint32_t L, double h, uint32_t count, hipStream_t s) {
    for (uint32_t k = 0; k < count; ++k) {
        ising_params p;
        std::memset(&p, 0, sizeof p);
        p.L = L;
        p.flags = ISING_PLAN_TWO_PASS;
        p.J = 1.0;
        p.h = h;
        p.T = 1.5 + 2.0 * (k + 0.5) / count;
        p.seed = 0x5eedull + k;
        p.p_up = 0.5;
        ising_ctx* c = nullptr;
        int rc = ising_create(&p, s, &c);
        if (rc != ISING_OK) return rc;
        set.ctxs.push_back(c);
        if ((rc = ising_reserve(c, 512)) != ISING_OK) return rc;
    }
    return ISING_OK;
}

int tune_device(int dev, Rates* out) {
    const uint32_t slots = engine_resident_slots(dev);
    if (slots == 0) return ISING_EDEVICE;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return ISING_EDEVICE;
    int rc = ISING_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = ISING_EDEVICE;
    Rates r;
    for (int b = 0; rc == ISING_OK && b < kBands; ++b) {
        const uint32_t L = kBandSide[b];
        const double site_sweeps = (double)L * L;  // per lattice and sweep
        // resident: two sweep counts (the larger about 4e9 site updates in
        // all), so the slope is the rate and the rest the fixed time per
        // lattice; stepped: about 1.5e9, in whole graph replays of 16 sweeps
        const uint64_t n_res = (uint64_t)std::min(512.0, std::max(4.0, std::round(4e9 / (site_sweeps * slots))));
        const uint64_t n_res0 = std::max<uint64_t>(1, n_res / 4);
        const uint64_t n_st =
            std::max<uint64_t>(16, (uint64_t)std::min(256.0, std::round(1.5e9 / (site_sweeps * slots))) / 16 * 16);
        for (int f = 0; rc == ISING_OK && f < 2; ++f) {
            const int c = 2 * b + f;
            TrialSet set;
            rc = make_set(set, L, f ? kTrialField : 0.0, slots, s);
            double t0 = 0.0, t1 = 0.0;
            if (rc == ISING_OK) rc = time_batch(set, n_res0, false, 0, s, e0, e1, &t0);
            if (rc == ISING_OK) rc = time_batch(set, n_res, false, 0, s, e0, e1, &t1);
            if (rc == ISING_OK) {
                // one lattice per workgroup: each time is one lattice's
                const double slope = std::max(t1 - t0, 1e-3 * t1) / (double)(n_res - n_res0);
                r.res[c] = site_sweeps / slope;
                r.res_fixed[c] = std::max(0.0, t0 - slope * (double)n_res0);
            }
            for (int ri = 0; rc == ISING_OK && ri < kRowChoices; ++ri) {
                double ns = 0.0;
                rc = time_batch(set, n_st, true, kRows[ri], s, e0, e1, &ns);
                if (rc == ISING_OK) r.st[c][ri] = site_sweeps * slots * n_st / ns;
            }
        }
    }
    if (rc == ISING_OK) {
        // one small lattice: the stepped plan's time per sweep is its launch
        TrialSet set;
        rc = make_set(set, 64, 0.0, 1, s);
        double ns = 0.0;
        if (rc == ISING_OK) rc = time_batch(set, 64, true, 0, s, e0, e1, &ns);
        if (rc == ISING_OK) r.floor_ns = ns / 64.0;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    if (rc != ISING_OK) return rc;
    r.tuned = true;
    *out = r;
    return ISING_OK;
}

}  // namespace

int batch_choose(ising_ctx* const* ctxs, const uint64_t* n, size_t count, int dev, BatchChoice* out) {
    const Rates r = rates_for(dev);
    const uint32_t slots = engine_resident_slots(dev);
    const uint32_t fslots = engine_fused_slots(dev);
    if (slots == 0 || fslots == 0) return ISING_EDEVICE;
    std::vector<double> t_res;
    double st[kRowChoices] = {0.0, 0.0, 0.0};
    uint64_t tiles[kRowChoices] = {0, 0, 0};
    uint64_t max_n = 0;
    bool fused = true;
    for (size_t k = 0; k < count; ++k) {
        if (n[k] == 0) continue;
        const ising_ctx* c = ctxs[k];
        const int cl = class_of(c->L, c->table);
        const double work = (double)c->L * c->L * (double)n[k];
        t_res.push_back(r.res_fixed[cl] + work / r.res[cl]);
        for (int ri = 0; ri < kRowChoices; ++ri) {
            st[ri] += work / r.st[cl][ri];
            if (multi_fused_supported(c->L)) tiles[ri] += multi_fused_tiles(c->L, kRows[ri]);
        }
        fused = fused && multi_fused_supported(c->L);
        max_n = std::max(max_n, n[k]);
    }
    BatchChoice ch{false, 0, 0.0, 0.0};
    ch.resident_ns = makespan(t_res, slots);
    double best = 0.0;
    for (int ri = kRowChoices - 1; ri >= 0; --ri) {  // ties go to the taller tiles
        double t = st[ri];
        if (fused && tiles[ri] > 0 && tiles[ri] < fslots) t *= (double)fslots / (double)tiles[ri];
        t = std::max(t, (double)max_n * r.floor_ns);
        if (ri == kRowChoices - 1 || t < best) {
            best = t;
            ch.rows = fused ? kRows[ri] : 0u;
        }
    }
    ch.stepped_ns = best;
    ch.stepped = !t_res.empty() && ch.stepped_ns < ch.resident_ns;
    *out = ch;
    return ISING_OK;
}

extern "C" {

int ising_batch_tune(int device, const char* cache_path, uint32_t flags, int* from_cache) {
    if (from_cache) *from_cache = 0;
    if (flags & ~ISING_TUNE_RETIME) return ISING_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) {
        (void)hipGetLastError();
        return ISING_EDEVICE;
    }
    if (device < 0 || device >= ndev || device >= kMaxDevices) return ISING_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return ISING_EDEVICE;
    if (!cache_path) cache_path = std::getenv("ISING_TUNE_CACHE");
    if (cache_path && !*cache_path) cache_path = nullptr;
    const std::string key = device_key(device);
    if (key.empty()) return ISING_EDEVICE;
    Rates r;
    if (cache_path && !(flags & ISING_TUNE_RETIME) && load_cache(cache_path, key, &r)) {
        std::lock_guard<std::mutex> g(g_mu);
        g_rates[device] = r;
        g_have[device] = true;
        if (from_cache) *from_cache = 1;
        return ISING_OK;
    }
    const int rc = tune_device(device, &r);
    if (rc != ISING_OK) return rc;
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_rates[device] = r;
        g_have[device] = true;
    }
    if (cache_path && !save_cache(cache_path, key, r)) return ISING_EIO;
    return ISING_OK;
}

int ising_batch_rates(int device, ising_batch_rate* out, size_t n, int* tuned, double* floor_ns) {
    if (device < 0 || device >= kMaxDevices || (!out && n)) return ISING_EINVAL;
    if (n < (size_t)kClasses) return ISING_EINVAL;
    const Rates r = rates_for(device);
    for (int c = 0; c < kClasses; ++c) {
        out[c].max_side = c / 2 < kBands - 1 ? kBandMax[c / 2] : ISING_MAX_L;
        out[c].field = (uint32_t)(c & 1);
        out[c].resident_per_workgroup = r.res[c];
        out[c].resident_fixed_ns = r.res_fixed[c];
        for (int ri = 0; ri < kRowChoices; ++ri) out[c].stepped[ri] = r.st[c][ri];
    }
    if (tuned) *tuned = r.tuned ? 1 : 0;
    if (floor_ns) *floor_ns = r.floor_ns;
    return ISING_OK;
}

int ising_batch_choice(ising_ctx* const* ctxs, const uint64_t* n_sweeps, size_t count, uint32_t* plan,
                       uint32_t* rows, double* predicted_ns) {
    if (!ctxs || !n_sweeps || count == 0) return ISING_EINVAL;
    int dev = -1;
    for (size_t k = 0; k < count; ++k) {
        if (!ctxs[k]) return ISING_EINVAL;
        if (dev < 0) dev = ctxs[k]->device;
        if (ctxs[k]->device != dev) return ISING_EINVAL;
    }
    if (hipSetDevice(dev) != hipSuccess) return ISING_EDEVICE;
    BatchChoice ch;
    const int rc = batch_choose(ctxs, n_sweeps, count, dev, &ch);
    if (rc != ISING_OK) return rc;
    if (plan) *plan = ch.stepped ? ISING_BATCH_STEPPED : ISING_BATCH_RESIDENT;
    if (rows) *rows = ch.rows;
    if (predicted_ns) {
        predicted_ns[0] = ch.resident_ns;
        predicted_ns[1] = ch.stepped_ns;
    }
    return ISING_OK;
}

}  // extern "C"
