// ctx.hpp -- the context object behind the opaque dugks_ctx handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/dugks.h"
#include "inst.hpp"

struct dugks_ctx {
    dugks_config cfg;
    int D = 0, Q = 0, esize = 0;
    long long nc = 0, ne = 0;
    void* met = nullptr;          // metric tables (device)
    void* inst_dev = nullptr;     // device copy of the instance parameters
    void* phi = nullptr;          // f-bar-plus scratch of the general kernels (device, lazily)
    double* partial = nullptr;    // per-block partial totals (device)
    double* totals_dev = nullptr; // reduced totals (device)
    int nblk_mom = 0;
    dugks::Inst<float> pf;
    dugks::Inst<double> pd;
    std::string err;
    int fast = 0;                 // fused-kernel variant selected at init (0 = none)
    int chunk = 0;                // planes marched per workgroup (0 = automatic)
    int n_cu = 0;                 // compute units of the device the context was created on
    int device = -1;              // ordinal of that device
    void* adj = nullptr;          // adjoint scratch (device, lazily)
    std::vector<double> faces_own[3]; // copies of custom face coordinates (cfg.faces points here)
    size_t adj_bytes = 0;
};

namespace dugks {
int fail(dugks_ctx* ctx, int code, const std::string& msg);
int hip_check(dugks_ctx* ctx, hipError_t e, const char* what);
int validate(const dugks_config* c, std::string& why);
// fused single-launch step for the configurations it supports
int setup_fast(dugks_ctx* ctx);
int fast_step(dugks_ctx* ctx, const void* fin, void* fout, const void* force, double t, hipStream_t st,
              bool* handled);
void release_fast(dugks_ctx* ctx);
void release_adjoint(dugks_ctx* ctx);
// address of the allocation-free adjoint's static scratch on the current
// device, looked up once per device (called by dugks_init)
void adjoint_static_setup();
}  // namespace dugks
