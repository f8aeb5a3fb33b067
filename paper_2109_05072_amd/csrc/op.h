// Host state of one operator handle (library-owned; device memory belongs to the caller).
#pragma once

#include <map>
#include <memory>
#include <string>
#include <utility>

#include "mfhex_internal.h"
#include "mg.h"

struct mfhex_op_s {
    mfhex_desc d{};           // copy of the description (vertex pointer cleared)
    mfhex::Basis1D basis{};
    int P = 0, Q = 0, g = 0;  // nodes / points per direction, factors per point
    int64_t N = 0, E = 0, NQ = 0;
    int device = 0;
    // views into the caller's workspace
    double *vert = nullptr;
    int32_t *offsets = nullptr;
    double *q64 = nullptr;
    float *q32 = nullptr;
    double *kappa = nullptr;
    double *wdet = nullptr;
    void *ebuf = nullptr;       // deterministic operators: element values [E][P^3][ncomp]
    int32_t *bad = nullptr;
    double *basis64 = nullptr;  // device basis block, FP64 and FP32
    float *basis32 = nullptr;
    bool kappa_set = false;
    std::map<std::pair<int, int>, mfhex::LaunchCfg> config;  // (prec, nvec) -> apply launch configuration
    std::unique_ptr<mfhex::MgHierarchy> mg;                  // p-multigrid levels (mfhex_mg_setup)
    std::string err;
    double *pinned = nullptr;  // small pinned host buffer for solver scalars
};

namespace mfhex {

// Workspace layout (byte offsets, 256-aligned); absent parts are SIZE_MAX.
struct Layout {
    size_t vert, offsets, q64, q32, kappa, wdet, ebuf, basis, bad, total;
};
Layout workspace_layout(const mfhex_desc &d, int64_t E, int P, int Q);

// Solver work layout for n nodes.
struct CgLayout {
    size_t r64, p64, ap64, r32, p32, ap32, partial, sc, hist, z64, dinv64, z32, dinv32, total;
};
constexpr int kHist = 8192;
CgLayout cg_layout(int64_t n);

int set_error(mfhex_op op, int code, const std::string &msg);
int fail_global(int code, const std::string &msg);  // failure of a call without a handle
// p-multigrid: one V-cycle z = M^-1 r on the fine operator; release of the hierarchy.
int mg_vcycle(mfhex_op op, const double *r, double *z, hipStream_t s);
void mg_release(mfhex_op op);
int check_hip(mfhex_op op, hipError_t e, const char *what);

// Internal apply: y (+)= A x on `s` with an explicit configuration.
// variant < 0 / chain <= 0: the handle's configuration for (prec, nvec).
// ebuf (optional): element-value buffer that makes this call deterministic (element values stored,
// then summed per node in a fixed order), in place of the operator's own.
int apply_impl(mfhex_op op, int prec, int nrhs, const void *x, void *y, hipStream_t s, bool zero, int variant = -1,
               int chain = 0, void *ebuf = nullptr);
int default_variant(const mfhex_op_s &op, int prec, int nvec);
bool valid_variant(const mfhex_op_s &op, int prec, int variant);
LaunchCfg config_for(const mfhex_op_s &op, int prec, int nvec);
// diag(M A M) (FP64, masked nodes 0) into d [N].
int diagonal_impl(mfhex_op op, double *d, hipStream_t s);
int default_chain(const mfhex_op_s &op);
int mode_of(const mfhex_op_s &op);

int cg_solve(mfhex_op op, const double *b, double *x, void *work, const mfhex_cg_opts *o, mfhex_cg_stats *st,
             double *rhist, hipStream_t s);
int tune(mfhex_op op, int prec, int nrhs, void *scratch, const char *cache_path, hipStream_t s);
void load_tune_cache(mfhex_op op);

}  // namespace mfhex
