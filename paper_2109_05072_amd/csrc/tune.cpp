// Autotuner for the fused apply: per (operator, precision, number of vectors)
// pick the launch variant (elements and threads per group) and, for the mass
// operator, the pipeline depth (element groups per thread group) by
// measurement.
//
// Every candidate is first checked against the default configuration on a
// random input (max-norm relative difference <= 1e-13 in FP64, 1e-5 in FP32;
// candidates only change the grouping of elements and lanes, so anything
// larger is a bug and the candidate is dropped), then timed with HIP events
// over repeated applies.  The winner is kept on the handle and appended to a
// text cache "<arch> kind quad p nvec prec variant depth", which later
// handles read from the file named by MFHEX_TUNE_CACHE.  This plays the role of the
// offline benchmark sweeps that select kernel variants per problem shape
// (Sec. 2, the MAGMA batched kernels chosen from tuning tables).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "blas.h"
#include "op.h"

namespace mfhex {

namespace {

std::string arch_name(int device)
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

}  // namespace

void load_tune_cache(mfhex_op op)
{
    const char *path = std::getenv("MFHEX_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    const std::string arch = arch_name(op->device);
    char line[256], a[64];
    while (std::fgets(line, sizeof line, f)) {
        int kind, quad, p, nvec, prec, epb, depth;
        if (std::sscanf(line, "%63s %d %d %d %d %d %d %d", a, &kind, &quad, &p, &nvec, &prec, &epb, &depth) != 8)
            continue;
        if (arch != a || kind != op->d.kind || quad != op->d.quad || p != op->d.p || !valid_variant(*op, prec, epb))
            continue;
        if (depth < 1 || depth > kMaxChain || (depth > 1 && mode_of(*op) != kMass)) continue;
        LaunchCfg c;
        c.variant = epb;
        c.chain = depth;
        op->config[{prec, nvec}] = c;
    }
    std::fclose(f);
}

int tune(mfhex_op op, int prec, int nrhs, void *scratch, const char *cache_path, hipStream_t s)
{
    if (!op) return set_error(nullptr, MFHEX_ERR_ARG, "null handle");
    if (!scratch || nrhs < 1) return set_error(op, MFHEX_ERR_ARG, "bad argument");
    if (prec == MFHEX_F32 && !op->q32) return set_error(op, MFHEX_ERR_STATE, "no FP32 data on this operator");
    const int nvec = nrhs * op->d.ncomp;
    const int64_t len = op->N * nvec;
    const size_t es = prec == MFHEX_F32 ? 4 : 8;
    // scratch: x (FP64 random, later cast in place for FP32), y_ref, y_test, partials
    char *w = static_cast<char *>(scratch);
    const size_t vb = ((size_t)len * 8 + 255) & ~size_t(255);
    double *x64 = reinterpret_cast<double *>(w);
    void *yref = w + vb, *ytest = w + 2 * vb;
    double *partial = reinterpret_cast<double *>(w + 3 * vb);
    double *out2 = partial + 2 * kRedBlocks;
    int c;
    auto cleanup = [&](int code) { return code; };
    const void *x = x64;
    if ((c = check_hip(op, launch_fill_uniform(x64, len, 5072, s), "fill kernel"))) return cleanup(c);
    if (prec == MFHEX_F32) {
        // FP32 copy of the input in the y_test slot first, then moved to the front
        if ((c = check_hip(op, launch_copy(x64, MFHEX_F64, ytest, MFHEX_F32, len, s), "copy kernel"))) return cleanup(c);
        if ((c = check_hip(op, hipMemcpyAsync(x64, ytest, len * es, hipMemcpyDeviceToDevice, s), "copy"))) return cleanup(c);
    }
    const int def = default_variant(*op, prec, nvec);
    if ((c = apply_impl(op, prec, nrhs, x, yref, s, true, def, default_chain(*op)))) return cleanup(c);
    std::vector<LaunchCfg> cand;
    const std::vector<int> depths = mode_of(*op) == kMass ? std::vector<int>{1, 2, 4} : std::vector<int>{1};
    for (int e = 0; e < kNumVariants; ++e)
        if (valid_variant(*op, prec, e))
            for (int d : depths) {
                LaunchCfg k;
                k.variant = e;
                k.chain = d;
                cand.push_back(k);
            }
    hipEvent_t e0, e1;
    if ((c = check_hip(op, hipEventCreate(&e0), "hipEventCreate"))) return cleanup(c);
    if ((c = check_hip(op, hipEventCreate(&e1), "hipEventCreate"))) return cleanup(c);
    // every candidate whose result agrees with the default is timed in three interleaved rounds of
    // ten back-to-back applies; the median of its rounds decides (candidates within a few percent
    // of each other change order from round to round)
    const int reps = 10, rounds = 3;
    const double tol = prec == MFHEX_F32 ? 1e-5 : 1e-13;
    std::vector<LaunchCfg> ok;
    for (const LaunchCfg &k : cand) {
        if ((c = apply_impl(op, prec, nrhs, x, ytest, s, true, k.variant, k.chain))) break;
        if ((c = check_hip(op, launch_relmaxdiff(ytest, yref, len, prec, partial, out2, s), "diff kernel"))) break;
        double h[2];
        if ((c = check_hip(op, hipMemcpyAsync(h, out2, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "copy"))) break;
        if ((c = check_hip(op, hipStreamSynchronize(s), "sync"))) break;
        if (h[0] <= tol * h[1]) ok.push_back(k);  // a wrong result rejects the candidate
    }
    std::vector<std::vector<float>> times(ok.size());
    for (int round = 0; round < rounds && !c; ++round) {
        for (size_t i = 0; i < ok.size() && !c; ++i) {
            const LaunchCfg &k = ok[i];
            if ((c = check_hip(op, hipEventRecord(e0, s), "event"))) break;
            for (int r = 0; r < reps && !c; ++r) c = apply_impl(op, prec, nrhs, x, ytest, s, true, k.variant, k.chain);
            if (c) break;
            if ((c = check_hip(op, hipEventRecord(e1, s), "event"))) break;
            if ((c = check_hip(op, hipEventSynchronize(e1), "event"))) break;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            times[i].push_back(ms);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (c) return cleanup(c);
    LaunchCfg best;
    best.variant = def;
    best.chain = default_chain(*op);
    float best_ms = 1e30f;
    for (size_t i = 0; i < ok.size(); ++i) {
        std::vector<float> t = times[i];
        std::sort(t.begin(), t.end());
        const float med = t[t.size() / 2];
        if (med < best_ms) {
            best_ms = med;
            best = ok[i];
        }
    }
    op->config[{prec, nvec}] = best;
    if (cache_path && *cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (f) {
            std::fprintf(f, "%s %d %d %d %d %d %d %d\n", arch_name(op->device).c_str(), op->d.kind, op->d.quad, op->d.p,
                         nvec, prec, best.variant, best.chain);
            std::fclose(f);
        }
    }
    return cleanup(MFHEX_OK);
}

}  // namespace mfhex
