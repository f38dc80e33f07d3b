// Autotuner of the level tiling (HPS_AUTOTUNE).
//
// Every tree level's products are cut into row tiles until the level launches at least a
// minimum number of workgroups (plan_panel).  Thin tiles fill the GPU at the top of the
// tree, where there are few nodes, but every extra tile gathers the node's input vector
// again; the best minimum depends on the grid, p, the precision and the device.  For one
// problem per launch the tuner measures it: the first build of an operator class builds
// the operator with each candidate minimum, times hps_solve (two warm-up solves, then the
// median of seven, HIP events on the build's stream), keeps the fastest, and remembers the
// choice for the process and, if the environment variable HPS_TUNE_FILE names a file, in
// that file (read again before every tuned build, rewritten after every measurement).
// Each tiling is tried with one launch per tree level and direction and, where the operator
// allows them, with composite level pairs (two levels per launch, hps_compose.hip).  The
// candidates only change how the same solve is multiplied out, so results differ from the
// untuned operator's by rounding only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hps_internal.h"

using namespace hps;

namespace {

constexpr int kCandidates[] = {1, 256, 1024, 4096};

struct Choice {
    int mwg = 0;
    int compose = 0;
    std::vector<std::pair<std::string, double>> us;   // candidate -> microseconds per solve (when measured here)
};

std::mutex g_tune_mu;
std::map<std::string, Choice> g_choices;

std::string class_key(const hps_grid *g, int flags, int ncomp) {
    char buf[128];
    std::snprintf(buf, sizeof(buf), "%dx%d_p%d_%s_%s%s", g->n1, g->n2, g->p, ncomp == 2 ? "complex" : "real",
                  (flags & HPS_FP32_IR) ? "fp32ir" : "fp64", (flags & HPS_UNIFORM_COEFFS) ? "_uniform" : "");
    return buf;
}

// Entries `"key": {"min_wg": N` of the tuning file (the format save() writes).
void load(const char *path) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    std::fclose(f);
    size_t pos = 0;
    while ((pos = text.find("\"min_wg\"", pos)) != std::string::npos) {
        // the key is the last quoted string before the '{' that opens this entry
        const size_t brace = text.rfind('{', pos);
        const size_t q1 = brace == std::string::npos ? std::string::npos : text.rfind('"', brace);
        const size_t q0 = q1 == std::string::npos || q1 == 0 ? std::string::npos : text.rfind('"', q1 - 1);
        const size_t colon = text.find(':', pos);
        if (q0 != std::string::npos && colon != std::string::npos) {
            const int v = std::atoi(text.c_str() + colon + 1);
            if (v > 0) {
                Choice &c = g_choices[text.substr(q0 + 1, q1 - q0 - 1)];
                c.mwg = v;
                // "compose": 1 within the same entry
                const size_t close = text.find('}', pos);
                const size_t cp = text.find("\"compose\"", pos);
                c.compose = 0;
                if (cp != std::string::npos && cp < close) {
                    const size_t c2 = text.find(':', cp);
                    if (c2 != std::string::npos) c.compose = std::atoi(text.c_str() + c2 + 1) ? 1 : 0;
                }
            }
        }
        pos += 8;
    }
}

void save(const char *path) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t k = 0;
    for (const auto &kv : g_choices) {
        std::fprintf(f, "  \"%s\": {\"min_wg\": %d, \"compose\": %d", kv.first.c_str(), kv.second.mwg,
                     kv.second.compose);
        if (!kv.second.us.empty()) {
            std::fprintf(f, ", \"us_per_solve\": {");
            for (size_t i = 0; i < kv.second.us.size(); ++i)
                std::fprintf(f, "%s\"%s\": %.2f", i ? ", " : "", kv.second.us[i].first.c_str(), kv.second.us[i].second);
            std::fprintf(f, "}");
        }
        std::fprintf(f, "}%s\n", ++k < g_choices.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

// Median time of seven hps_solve calls (after two warm-up calls) on stream st, in microseconds.
int time_solves(hps_op *op, hipStream_t st, double *us) {
    const int m = op->ncomp;
    double *body = nullptr, *u = nullptr;
    if (hipMalloc(&body, sizeof(double) * m * op->n_int) != hipSuccess ||
        hipMalloc(&u, sizeof(double) * m * op->N) != hipSuccess) {
        (void)hipGetLastError();
        if (body) (void)hipFree(body);
        hps_set_error("hipMalloc for the tuner's solves failed");
        return HPS_ENOMEM;
    }
    int rc = launch_zero(body, m * op->n_int, st);
    std::vector<hipEvent_t> ev(16, nullptr);
    for (hipEvent_t &e : ev)
        if (rc == HPS_OK && hipEventCreate(&e) != hipSuccess) rc = HPS_EDEVICE;
    for (int k = 0; k < 2 && rc == HPS_OK; ++k) rc = hps_solve(op, 1, body, nullptr, nullptr, u, st, nullptr);
    std::vector<float> t;
    for (int k = 0; k < 7 && rc == HPS_OK; ++k) {
        if (hipEventRecord(ev[2 * k], st) != hipSuccess) rc = HPS_EDEVICE;
        if (rc == HPS_OK) rc = hps_solve(op, 1, body, nullptr, nullptr, u, st, nullptr);
        if (rc == HPS_OK && hipEventRecord(ev[2 * k + 1], st) != hipSuccess) rc = HPS_EDEVICE;
    }
    if (rc == HPS_OK && hipStreamSynchronize(st) != hipSuccess) rc = HPS_EDEVICE;
    for (int k = 0; k < 7 && rc == HPS_OK; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) != hipSuccess) rc = HPS_EDEVICE;
        t.push_back(ms);
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipFree(body);
    (void)hipFree(u);
    if (rc == HPS_EDEVICE) hps_set_error("HIP event timing failed in the tuner");
    if (rc) return rc;
    std::sort(t.begin(), t.end());
    *us = 1e3 * t[t.size() / 2];
    return HPS_OK;
}

}  // namespace

int hps::tune_level_tiling(const hps_grid *grid, const hps_coeffs *coeffs, const hps_coeffs *coeffs_im,
                           double gamma_dt, int flags, hipStream_t st, int *mwg, int *compose) {
    const std::string key = class_key(grid, flags, coeffs_im ? 2 : 1);
    const char *path = std::getenv("HPS_TUNE_FILE");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (path && path[0]) load(path);
    auto it = g_choices.find(key);
    if (it != g_choices.end() && it->second.mwg > 0) {
        *mwg = it->second.mwg;
        *compose = it->second.compose;
        return HPS_OK;
    }
    // every tiling, with per-level sweeps and (where the operator allows them) with
    // composite level pairs
    Choice c;
    double best = 0.0;
    for (int comp = 0; comp < 2; ++comp)
        for (int cand : kCandidates) {
            hps_op *op = nullptr;
            TRY(build_op_tiled(grid, coeffs, coeffs_im, gamma_dt, flags, cand, comp, st, &op));
            if (comp && !op->composed) {   // no composites for this operator class
                hps_free(op);
                break;
            }
            double us = 0.0;
            const int rc = time_solves(op, st, &us);
            hps_free(op);
            if (rc) return rc;
            c.us.emplace_back(std::to_string(cand) + (comp ? "_pairs" : ""), us);
            if (c.mwg == 0 || us < best) {
                best = us;
                c.mwg = cand;
                c.compose = comp;
            }
        }
    g_choices[key] = c;
    if (path && path[0]) save(path);
    *mwg = c.mwg;
    *compose = c.compose;
    return HPS_OK;
}
