// gsr_ba.h -- device-side interface of the local bundle adjustment (FP64):
// sizes, the argument block its kernels share, and the launchers.
#pragma once
#include "gsr_internal.h"

namespace gsr {

// ---- local bundle adjustment (FP64) ----
constexpr int kBaMaxObs = 8;       // observation slots per landmark (lanes per landmark)
constexpr int kBaMaxFree = 20;     // free keyframes: reduced system of 6 * 20 + 1 unknowns
constexpr int kBaRecStride = 76;   // doubles per observation record (75 used)
constexpr int kBaLmStride = 12;    // doubles per landmark record (10 used)
constexpr int kBaAsmSplit = 4;     // workgroups (partial systems) per block of the reduced system

struct BaArgs {
    double *poses, *focal, *landmarks;
    const double *obs_uv;
    const int32_t *obs_cam, *free_slot, *slot_cam;
    const int32_t *rec_pos;   // record index of each observation slot in a free keyframe (keyframe-major), else -1
    const int2 *block_ab, *pairs;
    const uint32_t *block_off;
    double *obs_rec, *lm_rec, *S, *dc, *costs;
    double cx, cy, lambda;
    int K, M, F, D, nblk;
};

size_t ba_lds_bytes(int D);        // largest dynamic LDS of the solver's kernels
hipError_t ba_allow_lds(int D);
void launch_ba_iterations(const BaArgs &A, int iterations, hipStream_t st);

}  // namespace gsr
