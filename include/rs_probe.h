/*
 * rs_probe.h -- issue-rate probes of librs (measurement only, not part of the method).
 *
 * The direct sum of inverse ray-shooting (Thompson, Fluke, Barnes & Barsdell 2009, section 1
 * eq. 2; the 10-flop interaction of appendix A) is bound by the vector ALU: each ray-lens
 * interaction issues a fixed mix of float32 VOP2/VOP3 instructions and reciprocals.  Its
 * instruction-mix ceiling follows from the rates at which the GPU issues those instructions,
 * which these probes measure on the device the library runs on.
 */
#ifndef RS_PROBE_H
#define RS_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Instruction streams a probe can issue (every lane runs 16 independent register chains, so
 * throughput rather than latency is measured). */
typedef enum {
    RS_PROBE_FMAC_F32 = 0,   /* v_fmac_f32 (VOP2)                                            */
    RS_PROBE_FMA_F32 = 1,    /* v_fma_f32 (VOP3)                                             */
    RS_PROBE_MUL_F32 = 2,    /* v_mul_f32 (VOP2)                                             */
    RS_PROBE_RCP_F32 = 3,    /* v_rcp_f32 (transcendental unit)                              */
    RS_PROBE_MIX_13_1 = 4,   /* 13 v_fmac_f32 then 1 v_rcp_f32: the direct sum's per-pair mix */
    RS_PROBE_ADD_F64 = 5     /* v_add_f64 (the FP64 run combination)                          */
} rs_probe_op;

/*
 * Run the probe kernel for `op` on every compute unit at full occupancy, once to warm up and
 * once timed with HIP events on `stream` (synchronises the stream).
 *   lane_ops_per_s: host output, instructions issued per second summed over lanes (for the mix,
 *                   every instruction counts once, reciprocals included)
 *   seconds:        host output, nullable; the timed launch's duration
 * Nothing is allocated on the device.  Errors: RS_EINVAL (-1) for an unknown op or a NULL
 * output, RS_EDEVICE (-3) if a HIP call fails (text in rs_last_error).
 */
int rs_probe_issue_rate(int op, double *lane_ops_per_s, double *seconds, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RS_PROBE_H */
