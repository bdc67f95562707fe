// Autotuner of the Khatri-Rao core's workgroup tile.
//
// The FP32 and BF16x3 cores exist with two tile heights (64 or 128 rows of j1
// per workgroup, 256 columns of the unfolding either way).  The taller tile
// reuses each staged V2 (.) V3 fragment twice as often but holds twice the
// accumulators, which costs occupancy; which one wins depends on the ranks
// (tile padding of r1) and on R.  The tuner times both on the caller's own
// operands, on the caller's stream with HIP events, alternating the candidates
// over two rounds and keeping each one's fastest launch, and caches the winner
// per shape class: precision, output type, long-contraction variant, r1 in
// steps of 32, r2*r3 and R_pad in quarter octaves.  Each handle keeps its own
// cache and also consults one shared by every handle of the process (per
// device), so a shape class is timed once per process: later handles, possibly
// created while others load the GPU, take the first measurement.  The FP64 core
// has one tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

struct CoreTuner {
    std::map<std::array<int64_t, 6>, int> best;
};

CoreTuner* core_tuner_create() { return new CoreTuner(); }
void core_tuner_destroy(CoreTuner* T) { delete T; }

static int64_t quarter_octave(double x) { return (int64_t)std::floor(4.0 * std::log2(std::max(x, 1.0))); }

std::array<int64_t, 6> core_tune_key(int prec, int beta_f32, bool flush, int r1, int64_t r23, int64_t R_pad) {
    return {(int64_t)prec, (int64_t)beta_f32, (int64_t)flush, (int64_t)((r1 + 31) / 32), quarter_octave((double)r23),
            quarter_octave((double)R_pad)};
}

int core_tuner_lookup(const CoreTuner* T, const std::array<int64_t, 6>& key) {
    auto it = T->best.find(key);
    return it == T->best.end() ? 0 : it->second;
}

void core_tuner_store(CoreTuner* T, const std::array<int64_t, 6>& key, int tile) { T->best[key] = tile; }

// the process-wide cache: shape class and device -> tile
static std::mutex g_tune_mu;
static std::map<std::pair<int, std::array<int64_t, 6>>, int> g_tune_best;

static int shared_lookup(const std::array<int64_t, 6>& key) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_best.find({dev, key});
    return it == g_tune_best.end() ? 0 : it->second;
}

static void shared_store(const std::array<int64_t, 6>& key, int tile) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_best.emplace(std::make_pair(dev, key), tile);   // the first measurement stays
}

hipError_t time_candidates(const int* tiles, int ncand, const std::function<hipError_t(int)>& launch,
                           hipStream_t st, int* best) {
    constexpr int ROUNDS = 2;
    hipEvent_t ev[2 * ROUNDS * 2];
    const int nev = 2 * ROUNDS * ncand;
    for (int i = 0; i < nev; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) hipEventDestroy(ev[j]);
            return hipErrorOutOfMemory;
        }
    hipError_t e = hipSuccess;
    for (int rd = 0; rd < ROUNDS && e == hipSuccess; ++rd)
        for (int c = 0; c < ncand && e == hipSuccess; ++c) {
            const int k = 2 * (rd * ncand + c);
            hipEventRecord(ev[k], st);
            e = launch(tiles[c]);
            hipEventRecord(ev[k + 1], st);
        }
    if (e == hipSuccess) e = hipEventSynchronize(ev[nev - 1]);
    float tmin[2] = {1e30f, 1e30f};
    for (int rd = 0; rd < ROUNDS && e == hipSuccess; ++rd)
        for (int c = 0; c < ncand; ++c) {
            const int k = 2 * (rd * ncand + c);
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, ev[k], ev[k + 1])) != hipSuccess) break;
            tmin[c] = std::min(tmin[c], ms);
        }
    for (int i = 0; i < nev; ++i) hipEventDestroy(ev[i]);
    if (e != hipSuccess) return e;
    int b = 0;
    for (int c = 1; c < ncand; ++c)
        if (tmin[c] < tmin[b]) b = c;
    *best = tiles[b];
    // the output must hold the winner's result: run it again unless it ran last
    if (b != ncand - 1) e = launch(tiles[b]);
    return e;
}

hipError_t launch_core_tuned(CoreTuner* T, CoreArgs a, hipStream_t st, int* used) {
    if ((a.prec & 3) == 0 || a.r[0] < 1 || a.r[1] < 1 || a.r[2] < 1) {
        a.tile = core_tile_default(a.prec);
        *used = a.tile;
        return launch_core(a, st);
    }
    const auto key = core_tune_key(a.prec, a.beta_f32, a.R_pad > core_flush_span(), a.r[0],
                                   (int64_t)a.r[1] * a.r[2], a.R_pad);
    int known = core_tuner_lookup(T, key);
    if (!known && (known = shared_lookup(key)) != 0) core_tuner_store(T, key, known);
    if (known) {
        a.tile = known;
        *used = known;
        return launch_core(a, st);
    }
    const int tiles[2] = {64, 128};
    int best = 0;
    hipError_t e = time_candidates(
        tiles, 2,
        [&](int tile) {
            CoreArgs b = a;
            b.tile = tile;
            return launch_core(b, st);
        },
        st, &best);
    if (e != hipSuccess) return e;
    core_tuner_store(T, key, best);
    shared_store(key, best);
    *used = best;
    return hipSuccess;
}
