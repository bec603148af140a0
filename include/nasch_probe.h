/*
 * nasch_probe.h -- C ABI of libnasch_probe, the measurement companion of
 * libnasch: the sustained issue rate of the vector-ALU instructions the step
 * kernels consist of, on the current HIP device.
 *
 * The step of the model (van Zon & Ponce, Handout section "The
 * Nagel-Schreckenberg traffic model", rules 1-4) is integer-only, and with
 * temporal blocking the kernels that run it are bound by vector-ALU issue, not
 * by memory.  The performance analysis the paper asks for (Handout, "THE
 * ASSIGNMENT", item 6) therefore needs the ALU ceiling of the device, which
 * this library measures instead of assuming it.
 */
#ifndef NASCH_PROBE_H
#define NASCH_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Instruction kinds (the dominant instructions of the step kernels). */
#define NASCH_PROBE_BITOP3   0u /* v_bitop3_b32: any three-input bitwise function   */
#define NASCH_PROBE_ALIGNBIT 1u /* v_alignbit_b32: funnel shift of two words        */
#define NASCH_PROBE_BCNT     2u /* v_bcnt_u32_b32: population count plus addend     */
#define NASCH_PROBE_MUL_LO   3u /* v_mul_lo_u32: low word of a 32x32 product        */
#define NASCH_PROBE_MUL_HI   4u /* v_mul_hi_u32: high word of a 32x32 product       */
#define NASCH_PROBE_MAD_U64  5u /* v_mad_u64_u32: 32x32+64 -> 64 (Philox's multiply) */
#define NASCH_PROBE_DPP      6u /* v_mov_b32 with a DPP wave shift (cross-lane move) */
#define NASCH_PROBE_ADD      7u /* v_add_u32                                         */
#define NASCH_PROBE_XOR      8u /* v_xor_b32                                         */
#define NASCH_PROBE_SHIFT    9u /* v_lshlrev_b32 by a variable amount                */
#define NASCH_PROBE_LSHL_OR 10u /* v_lshl_or_b32: (a << s) | b                       */
#define NASCH_PROBE_PERM    11u /* v_perm_b32: byte select from two words           */
#define NASCH_PROBE_MUL_U24 12u /* v_mul_u32_u24: 24 x 24 -> low 32 bits             */
#define NASCH_PROBE_ADD_U64 13u /* v_lshl_add_u64: 64-bit add (address arithmetic)   */
#define NASCH_PROBE_MIN     14u /* v_min_u32                                         */
#define NASCH_PROBE_SUB     15u /* v_sub_u32                                         */
#define NASCH_PROBE_CNDMASK 16u /* v_cndmask_b32: select by a lane mask              */
#define NASCH_PROBE_AND_OR  17u /* v_and_or_b32: (a & b) | c                         */
#define NASCH_PROBE_BFI     18u /* v_bfi_b32: bitwise select (a & b) | (~a & c)     */
#define NASCH_PROBE_OR      19u /* v_or_b32                                          */
#define NASCH_PROBE_AND     20u /* v_and_b32                                         */
#define NASCH_PROBE_ADD3    21u /* v_add3_u32: a + b + c                             */
#define NASCH_PROBE_KINDS   22u

typedef struct {
    double ms;                 /* device time of the timed launch (HIP events)          */
    double wave_instructions;  /* wave64 instructions of the probed kind in that launch */
    double lane_ops_per_s;     /* wave_instructions x 64 / time                         */
    double sclk_hz;            /* shader clock during the launch: s_memtime cycles over */
                               /* s_memrealtime ticks (100 MHz), summed over blocks     */
} nasch_probe_result;

/*
 * Run `blocks` blocks of 256 threads (4 waves each), every lane executing
 * iters x 128 instructions of `kind` in 8 independent dependency chains, after
 * one short untimed launch.  Allocates and frees its own device memory and
 * stream on the current device; synchronises.  Returns 0, -1 for an invalid
 * argument, or minus the hipError_t of a failing HIP call.  Choose blocks to
 * fill the device (e.g. 8 per CU) and iters for a launch of some milliseconds.
 */
int nasch_probe_valu(uint32_t kind, uint32_t blocks, uint32_t iters, nasch_probe_result* res);

#ifdef __cplusplus
}
#endif
#endif /* NASCH_PROBE_H */
