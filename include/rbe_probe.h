/*
 * rbe_probe.h -- measurement support, not part of the method: an issue-rate
 * probe of the MI355X vector ALU. The roofline accounting of the near-field
 * and Fourier kernels states how many SIMD cycles one wave64 vector
 * instruction takes; this probe measures it for the instruction classes
 * those kernels are made of, so that the kernels' counted instruction rates
 * (rocprofv3 SQ_INSTS_VALU over the dispatch's clock, GRBM_GUI_ACTIVE) can
 * be set against what the hardware sustains for the same mix.
 *
 * rbe_probe_valu runs `blocks` workgroups of 256 threads on `stream`. Every
 * thread runs `iters` rounds of one instruction mix on registers (no memory
 * traffic inside the loop) and writes one float to out[block * 256 + thread]
 * (device; at least blocks * 256 floats) so that nothing is optimised away:
 *
 *   RBE_PROBE_FMA_F32   64 v_fma_f32 per round, 8 independent chains
 *   RBE_PROBE_MUL_ADD   64 FP32 multiplies and 64 adds per round, 8 chains
 *                       of a = a + b * c (FP32 multiply-add pairs, as the
 *                       near-field kernels' pair terms and Kahan sums issue)
 *   RBE_PROBE_LJ_BODY   four candidates of the LJ tile loop per round: FP32
 *                       displacement, r^2, the unsigned cutoff class, v_rcp_f32,
 *                       the masked LJ shape and its accumulation
 *   RBE_PROBE_RCP_F32   64 v_rcp_f32 per round, 8 independent chains
 *
 * *ms (host) receives the kernel's duration from HIP events around it; the
 * call synchronizes the stream. Returns RBE_OK, RBE_EINVAL (unknown kind,
 * blocks or iters below 1, null out or ms) or RBE_EDEVICE (a HIP call
 * failed; rbe_last_error(NULL) has the message).
 */
#ifndef RBE_PROBE_H
#define RBE_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { RBE_PROBE_FMA_F32 = 0, RBE_PROBE_MUL_ADD = 1, RBE_PROBE_LJ_BODY = 2, RBE_PROBE_RCP_F32 = 3 };

int rbe_probe_valu(int kind, int blocks, int iters, float *out, float *ms, void *stream);

#ifdef __cplusplus
}
#endif
#endif
