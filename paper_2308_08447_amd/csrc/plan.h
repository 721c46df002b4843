// plan.h -- host-side plan internals shared by the C ABI and the serving engine.
#pragma once

#include <array>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"

namespace dm {

// The transformed tensor of one mesh (geometry + cell size), computed once and
// shared by every plan of that mesh in the process.
struct Spectrum {
    Geometry g;
    double dx = 0, dy = 0, dz = 0;
    int kind = 0;         // 0 cell-averaged (Eq. 1), 1 point dipole (Eq. 8)
    float* K = nullptr;   // [6][Z1][X1][Y1]
    int device = 0;
    ~Spectrum();
    size_t bytes() const { return g.k_elems() * sizeof(float); }
};

// Looks the mesh up in the process-wide cache or computes it (FP64 on the GPU).
int get_spectrum(const Geometry& g, double dx, double dy, double dz, int kind, hipStream_t s,
                 std::shared_ptr<Spectrum>* out);
// Twiddle table of the current device (all lengths up to 4096), created once.
int device_twiddles(const float2** out);

// Bytes of the FFT workspace (S1 + S2 chunk buffer) and of the RK4 buffers.
// The three-kernel thin-mesh form is used by FP32 plans of supported sizes.
bool uses_xz(const Geometry& g, uint32_t flags);
size_t workspace_bytes(const Geometry& g, uint32_t flags);
size_t rk_bytes(const Geometry& g);
int s2_planes(const Geometry& g);

int dev_alloc(void** p, size_t bytes, const char* what);
// flags: plan flags (periodic axes and image count); 0 for an open mesh
int check_mesh(const demag_mesh* m, Geometry* g, uint32_t flags = 0);
int check_llg_params(const llg_params* prm, double dt, int32_t nsteps);

}  // namespace dm

struct demag_plan {
    std::shared_ptr<dm::Spectrum> spec;
    dm::Geometry g;
    double dx = 0, dy = 0, dz = 0;
    uint32_t flags = 0;
    int mf = 0;             // radix-16 passes: 0 FP32, 2 / 3 BF16 split-precision MFMA (terms)
    const float2* tw = nullptr;
    float2* S1 = nullptr;
    float2* S2 = nullptr;   // chunk buffer of xc kx planes; == S1 (xc = X1) when ny == 1
    bool xz = false;        // three-kernel form (T instead of S1 / S2)
    float2* T = nullptr;    // [3][Nz][G][ny][4] spectra of the three-kernel form
    int xc = 1;             // kx planes S2 holds
    int nch = 1;            // chunks the y/z stages are split into (>= ceil(X1 / xc))
    float* rk = nullptr;    // RK4 buffers (lazily allocated): H, A, B, acc, each 3 N floats
    float* hist = nullptr;  // DEMAG_EXTRAPOLATE_HD: ring of 5 step-start H_d fields (3 N each)
    int hist_n = 0;         // valid entries (<= 5)
    int hist_head = 0;      // slot of the newest entry
    double hist_dt = 0.0;   // step of the recorded trajectory
    int device = 0;
    int timing_cap = 0;     // per-stage event timing (demag_timing_enable)
    std::vector<hipEvent_t> ev[DEMAG_NSTAGES];
    int timing_n[DEMAG_NSTAGES] = {};
    int variant[5] = {1, 1, 1, 1, 1};   // tile-shape variant of each FFT stage
    // llg_step with nsteps >= 2: one RK4 step captured as a HIP graph on a
    // private stream and replayed; step_key identifies what the capture baked in
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t step_graph = nullptr;
    std::string step_key;
};

namespace dm {

// Creates a plan (workspace + shared spectrum) without the ABI's argument checks.
int create_plan(const demag_mesh* mesh, uint32_t flags, hipStream_t s, demag_plan** out);
void free_plan(demag_plan* p);
int ensure_rk(demag_plan* p);

// H_i = H_d(scale_i * M_i) for n plans, batching plans of equal transform
// lengths into shared launches (plans whose y/z stages run in one chunk);
// timing events are recorded only for single-plan calls.
int run_fields(demag_plan* const* plans, const float* const* M, float* const* H,
               const float* scale, int n, hipStream_t s);

struct LLGStep {            // one mesh in a batched RK4 step
    demag_plan* plan;
    float* m;
    llg_params prm;
    double dt;
    float* rk = nullptr;    // RK4 buffers (12 N floats); nullptr: the plan's own
};
// One classic RK4 step for every mesh in `steps` (batched launches).
int rk4_step_batch(const LLGStep* steps, int n, hipStream_t s);

}  // namespace dm
