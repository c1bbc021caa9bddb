// Launch-variant defaults and the autotuner of the hopping kernel (the
// batching form of the solver: the launch shape of each (precision, rhs
// count) is picked by timing, kept per gauge object).
#include <algorithm>
#include <cstdlib>
#include <utility>
#include <vector>

#include "common.h"

namespace rhmc {

void default_hop_variants(int (&v)[2][4]) {
    // index = order + 8 * batch + 24 * shape + 96 * tile
    // measured on MI355X at 48^3 x 12 (rhs classes 1, 2, 4, 8; every variant
    // timed): z-tiles of 4 or 6 planes (6: one XCD's share of z at Lz = 48)
    // with t inside a tile; rows staged in LDS except for eight right-hand
    // sides (128-site blocks); loads in batches of one to four hops; no rhs
    // tile (splitting four or eight rhs over two launches reads the links twice)
    const int fp64[4] = {68, 60, 36, 83};    // FP64-12 links (the default FP64 storage)
    const int fp32[4] = {36, 44, 36, 84};
    for (int k = 0; k < 4; ++k) {
        v[RHMC_PREC_FP64][k] = fp64[k];
        v[RHMC_PREC_FP32][k] = fp32[k];
    }
    if (const char* e = std::getenv("RHMC_HOP_VARIANT")) {
        const int f = std::abs(std::atoi(e)) % kHopVariants;
        for (auto& row : v)
            for (int& x : row) x = f;
    }
}

// Every variant is timed over a few launches; the fastest eight are timed
// again, three rounds of ten launches each, interleaved, and the one with the
// smallest median round wins (a single short pass picks among variants a few
// percent apart by noise).
rhmc_status tune_hop(rhmc_gauge* g, rhmc_prec prec, int nrhs, const void* in, void* out,
                     hipStream_t s) {
    const int cls = nr_class(nrhs);
    const size_t n = (size_t)3 * g->lat.Vh;
    // each timed launch between its own pair of events: in a solve every
    // hopping launch sits between other kernels, and back-to-back launches of
    // one variant (each starting while the previous one's output stores
    // drain) rank the variants differently
    constexpr int kMaxReps = 10;
    hipEvent_t ev[2 * kMaxReps] = {};
    for (int i = 0; i < 2 * kMaxReps; ++i) {
        const hipError_t ce = hipEventCreate(&ev[i]);
        if (ce != hipSuccess) {
            for (int k = 0; k < i; ++k) hipEventDestroy(ev[k]);
            RHMC_HIP_TRY(ce);
        }
    }
    std::vector<std::pair<float, int>> pass1;
    // median time of `reps` (<= kMaxReps) launches of variant v after `warm`
    // untimed ones (ms per launch)
    auto time_variant = [&](int v, int warm, int reps, float* ms_out) -> hipError_t {
        hipError_t err = hipSuccess;
        auto launch = [&]() {
            if (prec == RHMC_PREC_FP64) {
                DslashArgs<double2> a{};
                a.g = g->lat.geom;
                a.out_par = 1;
                a.nrhs = nrhs;
                a.variant = v;
                for (int r = 0; r < nrhs; ++r) {
                    a.in[r] = reinterpret_cast<const double2*>(in) + r * n;
                    a.out[r] = reinterpret_cast<double2*>(out) + r * n;
                }
                err = launch_fp64_op(g, a, kModeD, s);
            } else {
                DslashArgs<float2> a{};
                a.g = g->lat.geom;
                a.out_par = 1;
                a.nrhs = nrhs;
                a.variant = v;
                a.paired = paired_f32(nrhs);
                for (int r = 0; r < nrhs; ++r) {
                    a.in[r] = reinterpret_cast<const float2*>(in) + f32_offset(a.paired, r, 0, n);
                    a.out[r] = reinterpret_cast<float2*>(out) + f32_offset(a.paired, r, 0, n);
                }
                err = launch_fp32_op(g, a, kModeD, s);
            }
        };
        for (int w = 0; w < warm && err == hipSuccess; ++w) launch();
        for (int w = 0; w < reps && err == hipSuccess; ++w) {
            err = hipEventRecord(ev[2 * w], s);
            if (err == hipSuccess) launch();
            if (err == hipSuccess) err = hipEventRecord(ev[2 * w + 1], s);
        }
        if (err == hipSuccess) err = hipEventSynchronize(ev[2 * reps - 1]);
        float t[kMaxReps];
        for (int w = 0; w < reps && err == hipSuccess; ++w) err = hipEventElapsedTime(&t[w], ev[2 * w], ev[2 * w + 1]);
        if (err == hipSuccess) {
            std::sort(t, t + reps);
            *ms_out = t[reps / 2];
        }
        return err;
    };
    hipError_t err = hipSuccess;
    for (int v = 0; v < kHopVariants && err == hipSuccess; ++v) {
        float ms = 0.f;
        err = time_variant(v, 2, 5, &ms);
        pass1.push_back({ms, v});
    }
    const int cur_v = g->hop_variant[prec][cls];
    int best_v = cur_v;
    if (err == hipSuccess) {
        std::sort(pass1.begin(), pass1.end());
        // the fastest eight of the first pass, and the current variant (the
        // measured default unless a caller pinned another): five launches can
        // misorder variants a few per cent apart
        std::vector<int> cand;
        for (int c = 0; c < std::min<int>(8, (int)pass1.size()); ++c) cand.push_back(pass1[c].second);
        if (std::find(cand.begin(), cand.end(), cur_v) == cand.end()) cand.push_back(cur_v);
        const int nc = (int)cand.size();
        std::vector<std::vector<float>> rounds(nc);
        for (int r = 0; r < 3 && err == hipSuccess; ++r)
            for (int c = 0; c < nc && err == hipSuccess; ++c) {
                float ms = 0.f;
                err = time_variant(cand[c], 2, 10, &ms);
                rounds[c].push_back(ms);
            }
        float best = 1e30f, cur = 1e30f;
        for (int c = 0; c < nc && err == hipSuccess; ++c) {
            std::sort(rounds[c].begin(), rounds[c].end());
            const float med = rounds[c][rounds[c].size() / 2];
            if (cand[c] == cur_v) cur = med;
            if (med < best) {
                best = med;
                best_v = cand[c];
            }
        }
        // a variant replaces the current one only if it is more than 3% faster:
        // tuned inside a solve, variants 1-2% apart swap places from run to run
        if (err == hipSuccess && cur <= 1.03f * best) best_v = cur_v;
    }
    for (int i = 0; i < 2 * kMaxReps; ++i) hipEventDestroy(ev[i]);
    RHMC_HIP_TRY(err);
    g->hop_variant[prec][cls] = best_v;
    g->hop_tuned[prec][cls] = 1;
    return RHMC_OK;
}

}  // namespace rhmc
