/*
 * mppi_ceilings.h — measured hardware ceilings beside the MPPI kernels
 * (libmppi_ceilings.so).  Not part of the MPPI method: these kernels give the
 * benchmark its measured issue-rate and latency floors, next to the MI355X
 * datasheet figures, so that each MPPI kernel's position can be stated
 * against what the chip actually sustains.
 *
 * Conventions (as in mppi.h): d_ pointers are device memory, the rest host;
 * every call runs on the given HIP stream (not NULL: graph capture needs a
 * created stream), waits for its own work and returns the average time of
 * one launch (or graph replay) in *us_out, measured with HIP events on that
 * stream around `reps` launches after one untimed warm-up.  Errors: -1 for
 * an invalid argument, -3 when a HIP call fails (the HIP error string is in
 * mppi_ceiling_last_error()).
 */
#ifndef MPPI_CEILINGS_H
#define MPPI_CEILINGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Independent-chain VALU loop: `blocks` workgroups of 256 threads, each
 * thread running `iters` loop trips of 8 independent chains of one
 * instruction kind:
 *   mode 0: v_fma_f32 (binary32 fused multiply-add; 8 lane-ops per trip);
 *   mode 1: 8 v_fma_f32 and 2 v_exp_f32 per trip (do transcendentals issue
 *           beside FMAs, or in the same slots?);
 *   mode 2: v_exp_f32 only (8 per trip);
 *   mode 3: v_mad_u64_u32 (32 x 32 -> 64-bit multiply-add, Philox's product;
 *           8 per trip);
 *   mode 4: 32-bit integer v_xor_b32 and v_add_u32 (16 per trip).
 * d_sink: blocks * 256 floats, written so that nothing is optimised away.
 * *lane_ops_out: VALU lane-instructions the loop body issues per launch
 * (blocks * 256 * iters * instructions per trip). */
int mppi_ceiling_valu(int32_t mode, int32_t blocks, int32_t iters, int32_t reps, float* d_sink,
                      void* hip_stream, double* us_out, double* lane_ops_out);

/* One wave's dependent T-step chain, the floor of any rollout of horizon T:
 * each of 64 lanes advances a forward-Euler double integrator (state 4,
 * control 2) through T steps, reading its two controls of step t from
 * d_eps[t][2][64] (binary32, device, 128 T floats) and accumulating a
 * quadratic cost; the loads do not depend on the state, so only the
 * arithmetic chain and one memory round trip are exposed (T <= 256).
 * d_out: 64 floats. */
int mppi_ceiling_chain(int32_t T, int32_t reps, const float* d_eps, float* d_out,
                       void* hip_stream, double* us_out);

/* Graph replay of `kernels` empty one-wave kernels in stream order (the shape
 * of one MPPI iteration: noise, rollout, update), `iterations` times per
 * graph; *us_out: average time of one replay.  The launch floor of a captured
 * iteration sequence. */
int mppi_ceiling_graph(int32_t kernels, int32_t iterations, int32_t reps, void* hip_stream,
                       double* us_out);

const char* mppi_ceiling_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MPPI_CEILINGS_H */
