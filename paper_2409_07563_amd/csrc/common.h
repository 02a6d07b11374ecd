// Internal definitions shared by the HIP translation units of libmppi.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mppi.h"

namespace mppi {

constexpr int kWave = 64;

// Model and cost constants as the kernels see them: passed by value as a
// kernel argument, so every field is wave-uniform (SGPR) and array pointers
// point into the context's workspace.
struct DevParams {
  // integration
  float dt, half_dt, sixth_dt;
  // bicycle
  float inv_wheelbase;
  // quadrotor
  float inv_mass, gravity;
  float inertia[3], inv_inertia[3];
  // MLP residual: operand packs of the MFMA tiles (mlp.h)
  int mlp_hidden;
  const float* mlp;      // forward pack
  const float* mlp_bwd;  // transposed-weight pack of the adjoint
  // cost
  float w[32];
  const float* ref;
  int nseg;
  int ncirc;
  // Read-only cost data that the rollout kernel stages into LDS (one float4
  // array, `stage_words4` long):
  //   circle grid at float4 offset 0: ncell+1 uint32 list offsets padded to
  //   grid_off4 float4s, then the entries (cx, cy, r2, 0), each circle listed
  //   in every cell its (slightly inflated) bounding box touches;
  //   spline at float4 offset spline_coef4: nseg coefficient rows (c0..c3),
  //   then the nseg+1 knots from float4 offset spline_knot4.
  const float4* stage;
  int stage_words4;
  int grid_nx, grid_ny, grid_off4;
  float grid_x0, grid_y0, grid_inv_cell;
  int spline_coef4, spline_knot4;
  int map_w, map_h;
  float map_x0, map_y0, map_res, map_inv_res;
  const float* costmap;   // [map_h][map_w]
  // A costmap holding at most two distinct values (an occupancy map: free /
  // obstacle) is also staged losslessly as a bitmap: bit iy*map_w + ix of the
  // uint32 words at float4 offset map_bits4 of the stage selects map_v1 (set)
  // or map_v0; map_bits4 < 0 when the map is read from memory instead.
  int map_bits4;
  float map_v0, map_v1;
  // importance-sampling term of a step: sum_j is_coef[j] (v_j - u_j/2) u_j with
  // is_coef[j] = lambda / sigma_j^2 (added to the running cost when importance)
  int importance;
  float is_coef[MPPI_MAX_CONTROL];
  // nested cosines ahead of each running cost (a pure compute load)
  int cosines;
  // sampling options: samples k < n_plain are drawn around u, the others
  // around zero; per-step importance coefficients lambda / sigma_{t,j}^2
  // ([T][m], null: is_coef for every step) and noise deviations ([T][m],
  // null: the configuration's sigma)
  int n_plain;
  const float* is_coef_t;
  const float* sigma_t;
  int mean_sample;  // sample 0 drawn without noise
  // MLP residual in BF16 mode: the bfloat16 weight pack (mlp.h), else null
  const uint4* mlp_bf;
};

// Largest circle grid the rollout kernel stages into LDS.
constexpr int kMaxGridBytes = 64 * 1024;

struct Sigma8 { float v[MPPI_MAX_CONTROL]; };

// The next iteration's noise, drawn by extra workgroups of a rollout or update
// launch into the other buffer with word *word_in + 1 (word_in: the word of
// the buffer the launch reads), which they record in *word_out; kblocks is
// filled in by the launcher.
struct NoiseJob {
  uint32_t key0, key1, instance;
  const uint32_t* word_in;
  uint32_t* word_out;
  int K, T, TM;
  Sigma8 sigma;
  float* eps;
  int64_t ldk;
  const float* sigma_t;
  int mean_sample;
  int calls;
  int kblocks;
};

// Workgroups of `threads` threads that draw a NoiseJob: kblocks sample blocks
// times the Philox call groups (fills job->kblocks).
inline int noise_job_blocks(NoiseJob* job, int threads) {
  job->kblocks = (job->K + threads - 1) / threads;
  const int ncall = (job->TM + 3) / 4;
  return job->kblocks * ((ncall + job->calls - 1) / job->calls);
}

// Device-side scalars of a context.
struct DevState {
  float stats[4];     // rho, eta, free energy, 1/sum w^2
  int32_t status;     // MPPI_OK or MPPI_ENUMERIC
  uint32_t iteration; // Philox iteration word of the next sampling
  float wz;           // weight of the samples drawn around zero (0 when none)
  int32_t pad;
};

// One instance of a batch, as the batched kernels read it (device memory).
struct BatchInst {
  DevParams p;
  const float* x0;
  float* u;
  float* eps;
  float* S;
  int32_t* crashes;  // null unless crash counting
  int64_t ldk;
  int K, T, TM;
  float lambda, inv_lambda;
  float step;  // step size gamma of the update
  uint32_t key0, key1, instance;
  Sigma8 sigma;
  float* e;  // unnormalised weights exp(-(J_k - rho)/lambda) [ldk]
  DevState* st;
  // the one-launch form's tile partials: weighted noise rows [ntile][TM]
  // and (minimum, sum e, sum e^2, sum e over the zero-mean samples) [ntile]
  float* tile_part;
  float4* tile_stat;
};

// Work lists of the batched kernels (host-built, device-resident):
//   sample tiles (instance, block of `tile` samples), longest horizon first;
//   row tiles (instance, block of gemv_rows_per_block() rows of the update).
// The tile size is a launch parameter (64, 128 or 256 samples, one thread
// each; the autotuner picks it); kBatchMinTile sizes the tile table.
constexpr int kBatchMaxTile = 256, kBatchMinTile = 64;

// Most tiles of one instance in the one-launch batch form (K <= 65536).
constexpr int kOneLaunchMaxTiles = 256;

// Segment-parallel reverse pass: the most 16-sample tiles of nonzero weight it
// takes (also at most 1280 / units; its scratch is sized for that many),
// and the default bound.
constexpr int kAdjointTilesMax = 128, kAdjointTilesDefault = 64;
struct BatchPlan {
  const BatchInst* insts;
  const int2* sample_tiles;
  int n_sample_tiles;
  int tile;
  const int2* row_tiles;
  int n_row_tiles;
  int n_inst;
  size_t rollout_lds;
  size_t max_tm_bytes;  // largest T * m of an instance, in bytes (the shift's LDS)
  // the one-launch form: its sample tiles of kBatchMaxTile (longest horizon
  // first; one workgroup each) and the per-instance tile counters
  const int2* fused_items;
  int n_fused_items;
  uint32_t* done;
};

// ---- host launchers (one translation unit each) ---------------------------
// The iteration word is *d_iteration + iteration when d_iteration is given
// (read on the device at run time), else iteration.
// calls: Philox calls per thread (1, 2 or 4; the values do not depend on it)
// d_sigma_t (optional, device [T][m]): per-step deviations replacing sigma;
// mean_sample: eps[.][.][0] = 0.
hipError_t launch_noise(uint64_t seed, const uint32_t* d_iteration, uint32_t iteration,
                        uint32_t instance, int K, int T, int m, const float* sigma,
                        float* d_eps, int64_t ldk, hipStream_t stream, int calls = 1,
                        const float* d_sigma_t = nullptr, bool mean_sample = false,
                        uint32_t* d_word_out = nullptr);
hipError_t launch_noise_tables(float* d_r, float* d_c, float* d_s, hipStream_t stream);

// Returns hipErrorInvalidValue when the (dynamics, integrator, cost)
// combination has no kernel.
// lanes: 1 lane per sample, or 4, 8 or 16 where the grouped kernel exists
// (bicycle, RK4: rollout_quad_available).
bool rollout_quad_available(uint32_t dynamics, uint32_t integrator);
// block: threads per workgroup, 64, 128 or 256
hipError_t launch_rollout(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                          bool accurate_trig, int lanes, const DevParams& p, const float* d_x0,
                          const float* d_u, const float* d_eps, int64_t ldk, int K, int T,
                          float* d_S, int32_t* d_crashes, hipStream_t stream, int block = 64,
                          const NoiseJob* next = nullptr);
bool rollout_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost);

// The time-parallel form of (a2) (rollout_scan.hip): the bicycle with RK4, a
// sample's horizon spread over the 16 lanes of a DPP row (T <= 256); block:
// threads per workgroup (64, 128, 256).
// lanes: per sample, 16 (one DPP row) or 32 (two)
bool rollout_scan_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost, int T,
                            int lanes = 16);
hipError_t launch_rollout_scan(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                               bool accurate_trig, const DevParams& p, const float* d_x0,
                               const float* d_u, const float* d_eps, int64_t ldk, int K, int T,
                               float* d_S, int32_t* d_crashes, hipStream_t stream, int block,
                               const NoiseJob* next = nullptr, int lanes = 16);

// The split form of (a2) (split.hip): a dynamics kernel writes the states
// x_1..x_T of every sample to d_traj ([T][traj_words][ldk], the state then,
// for the costmap cost, the compensation of the position), a cost kernel
// evaluates all steps in parallel.  lanes: 1, or 4 (bicycle, RK4); block:
// dynamics threads per workgroup (64, 128, 256); waves: cost waves per 64
// samples, a power of two up to kSplitMaxWaves * kSplitMaxChunks (up to 16 in
// one workgroup, more as chunks of 16 whose partial sums go to d_part:
// kSplitMaxChunks * ldk floats, then as many ints).
constexpr int kSplitMaxWaves = 16, kSplitMaxChunks = 8;
bool rollout_split_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost);
int split_traj_words(uint32_t dynamics, uint32_t cost);
hipError_t launch_rollout_split(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                                bool accurate_trig, int lanes, const DevParams& p,
                                const float* d_x0, const float* d_u, const float* d_eps,
                                int64_t ldk, int K, int T, float* d_traj, float* d_part,
                                float* d_S, int32_t* d_crashes, hipStream_t stream, int block,
                                int waves);
// LDS bytes the rollout kernel stages (cost data + the nominal controls).
size_t rollout_lds_bytes(uint32_t dynamics, uint32_t cost, int stage_words4, int T);
constexpr size_t kMaxRolloutLds = 160 * 1024;

int gemv_rows_per_block();
// The differentiation tape of gradient mode (device pointers; u null: none):
// the weights step records u and the iteration word of the update in slot
// *count (if below cap) and advances the count (cap + 1 marks an overflow).
struct TapeRef {
  const float* u = nullptr;
  int TM = 0;
  float* tape_u = nullptr;
  uint32_t* tape_word = nullptr;
  int32_t* count = nullptr;
  int cap = 0;
};

// step: the step size gamma of u += gamma sum_k w_k (v_k - u) (1 for
// Algorithm 1); samples k >= n_plain were drawn around zero (n_plain = K:
// none); tape: see TapeRef.
// Samples up to which the single-pass update exists.
constexpr int kOnePassMaxK = 16384;
// Samples per workgroup of the chunked update's weights step.
constexpr int kWChunk = 2048;

hipError_t launch_softmin_update(const float* d_S, const float* d_eps, int64_t ldk, int K,
                                 int TM, float lambda, float step, float* d_e, float* d_u,
                                 DevState* d_state, hipStream_t stream, int n_plain,
                                 const TapeRef& tape = TapeRef{}, const NoiseJob* next = nullptr);
// Steps (a3)-(a6) for a single instance of any size (no gradient mode): the
// weights step spread over ceil(K / kWChunk) workgroups (with a next-noise job
// the same launch draws the next iteration's noise), then the rows;
// d_part holds ceil(K / kWChunk) float4.
hipError_t launch_update_chunked(const float* d_S, const float* d_eps, int64_t ldk, int K,
                                 int TM, float lambda, float step, float* d_e, float4* d_part,
                                 float* d_u, DevState* d_state, hipStream_t stream, int n_plain,
                                 const NoiseJob* next);
// Steps (a3)-(a6) in one launch for a single instance with K <= 16384 (one
// workgroup per row computes the weights itself), optionally drawing the next
// iteration's noise too.
hipError_t launch_update_one_pass(const float* d_S, const float* d_eps, int64_t ldk, int K,
                                  int TM, float lambda, float step, float* d_u,
                                  DevState* d_state, hipStream_t stream, int n_plain,
                                  const NoiseJob* next);
hipError_t launch_set_iteration(DevState* d_state, uint32_t iteration, hipStream_t stream);
hipError_t launch_weights(const float* d_S, int K, float lambda, const DevState* d_state,
                          float* d_w, hipStream_t stream);

// MLP residual dynamics and the checkpointing forward (rollout_tiles.hip)
bool rollout_tiles_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost, int hidden);
// waves: waves per 16-sample tile: 1, or the MLP split over 2 (H = 32, 64)
// or 4 (H = 64) waves; hipErrorInvalidValue for other combinations
hipError_t launch_rollout_tiles(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                                bool accurate_trig, const DevParams& p, const float* d_x0,
                                const float* d_u, const float* d_eps, int64_t ldk, int K, int T,
                                float* d_S, float* d_ckpt, int ckpt_every, hipStream_t stream,
                                int waves = 1);

// The adjoint (adjoint.hip).  Scratch: byte offsets inside one device region.
struct AdjointScratch {
  size_t gk, part, offs, meta, list, partial, pre, tp, total;
  int64_t ngp;  // floats per partial-gradient row
};
int adjoint_grad_len(uint32_t dynamics, int hidden);
// TM = T * m: room for the dL/du columns of the partial rows
AdjointScratch adjoint_scratch_layout(int K, int ngrad, int hidden, int ckpt_every, int TM);
size_t adjoint_lds_bytes(int hidden, int ckpt_every, bool bf16 = false);
// accumulate: d_grad += the gradient (else d_grad = it); d_G_acc (optional):
// d_G_acc += sum_k a_k dJ_k/du (may be d_G itself: the update happens after
// every read of d_G, in stream order).  tp_tiles: the segment-parallel
// reverse pass when at most that many tiles hold listed samples (0: never;
// capped at 128, at 1280 / units and at the context's tile count).
hipError_t launch_adjoint(const DevParams& p, bool accurate_trig, int hidden, const float* d_G,
                          const float* d_u, const float* d_eps, int64_t ldk, int K, int T,
                          const float* d_e, float lambda, float step, const float* d_ckpt,
                          int ckpt_every, char* d_scratch, const AdjointScratch& s, int ngrad,
                          float* d_grad, hipStream_t stream, int waves = 1,
                          bool accumulate = false, float* d_G_acc = nullptr,
                          int tp_tiles = 0);
hipError_t launch_weights_only(const float* d_S, int K, float lambda, float* d_e,
                               DevState* d_scratch_state, hipStream_t stream);
// The differentiation tape: start over (count = 0).
hipError_t launch_tape_reset(int32_t* d_count, hipStream_t stream);
// u[t] <- u[min(t + steps, T - 1)] (fill 0) or 0 past the horizon (fill 1)
hipError_t launch_shift(float* d_u, int T, int m, int steps, int fill, hipStream_t stream);
hipError_t launch_batch_shift(const BatchPlan& b, int steps, int fill, hipStream_t stream);

hipError_t launch_batch_noise(const BatchPlan& b, hipStream_t stream);
hipError_t launch_batch_rollout(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                                bool accurate_trig, bool count, const BatchPlan& b,
                                hipStream_t stream);
hipError_t launch_batch_update(const BatchPlan& b, hipStream_t stream);
// One launch per iteration for a whole batch: every sample tile
// (kBatchMaxTile samples) draws its noise, rolls out and leaves its softmin
// partials; the workgroup that completes an instance's last tile updates it.
hipError_t launch_batch_one_launch(uint32_t dynamics, uint32_t integrator, uint32_t cost,
                                   bool accurate_trig, bool count, const BatchPlan& b,
                                   hipStream_t stream);
bool batch_one_launch_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost);
// One iteration of a single double-integrator instance (forward Euler, the
// quadratic cost) in one time-parallel launch; K <= 4096, T <= 256.  b: the
// instance's descriptor with tile partials for ceil(K / 16) tiles of 16
// samples; d_done: its zeroed completion counter.
bool di_iteration_supported(uint32_t dynamics, uint32_t integrator, uint32_t cost, int K, int T);
int di_iteration_tiles(int K);
hipError_t launch_di_iteration(const BatchInst& b, uint32_t* d_done, hipStream_t stream);
hipError_t launch_batch_set_iteration(const BatchPlan& b, uint32_t iteration, hipStream_t stream);

// ---- wave / block reductions ------------------------------------------------
__device__ inline float wave_min(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

}  // namespace mppi
