// Kernel-side argument blocks and launchers of liblead (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/lead.h"
#include "lead_args.hpp"
#include "lead_device.hpp"

namespace lead {

constexpr int kMaxWorkgroup = 256;   // threads per workgroup
constexpr uint32_t kNoOwn = 0xFFFFFFFFu;

struct SyndArgs {
    const uint64_t *err;
    uint64_t *synd;
    const int32_t *view;
    int64_t shots, err_words, synd_words;
    int32_t N, D2, r, m;
    uint64_t mask[kMaxChecks];
};

// Plain (one launch per round) decode state kept in HBM.
struct RoundArgs {
    DecodeArgs d;
    float *S;                  // [shots][D2][N] variable sums
    float *cst;                // [shots][r][4][N] check states (m1, m2, am, q)
    const float *lamp;         // [shots][n] lambda'
    int32_t *status;           // [shots][4] done, converged, iterations, unused
    int32_t *active;           // device counter of shots still iterating
    int32_t phase;             // 0 init, 1 round, 2 finalize
    int32_t round;             // 1-based round index for phase 1
};

size_t decode_lds_bytes(int D, int wg, int spw, int n);
int workgroup_size(int N, int spw);

// ev (split path only, may be null): events recorded before the Phase 1
// kernel, between the two kernels, and after the Phases 2-3 kernel.
hipError_t launch_decode(int D, int rmax_needed, const DecodeArgs &a, const LocalArgs &w, bool split,
                         hipStream_t s, hipEvent_t *ev = nullptr);
hipError_t launch_round(int D, int rmax_needed, const RoundArgs &a, hipStream_t s);
hipError_t launch_reset_counter(int64_t *counter, hipStream_t s);
// Clears n int64 words with a fill kernel (no memset node under capture).
hipError_t launch_clear_i64(int64_t *p, int n, hipStream_t s);
hipError_t launch_syndrome(const SyndArgs &a, hipStream_t s);
bool kernel_supported(int D, int r);
int local_waves_per_cu(int D, int pm);

}  // namespace lead
