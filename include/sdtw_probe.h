/*
 * Measurement probe behind the VALU roof of the sDTW benchmark (libsdtw_probe.so,
 * separate from libsdtw.so; not part of the alignment path).
 *
 * The cell update of section 2.3 Eq. 1 is two 32-bit VALU instructions on the
 * int16 path (v_min3_u32, v_sad_u32) and three on the float32 path
 * (v_sub_f32, v_min3_u32, v_add_f32 with |.|).  The roof converts cell updates
 * into SIMD cycles with the issue rate of each instruction kind, which this
 * probe measures.
 */
#ifndef SDTW_PROBE_H
#define SDTW_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Launch 4 x CUs x waves_per_simd one-wave workgroups, each reserving
 * 1 / (4 x waves_per_simd) of a CU's 160 KiB of LDS (so every SIMD holds
 * waves_per_simd of them), each running iters x 16 x chains instructions of
 * one kind in `chains` independent dependency chains:
 *   kind 0 v_min3_u32, 1 v_sad_u32, 2 v_sub_f32, 3 v_add_f32 |a| + d,
 *   4 v_add_u32.
 *   chains 1, 2 or 4; waves_per_simd 1..8; iters >= 1.
 *   out_dev  device buffer of 4 x CUs x waves_per_simd x 64 uint32 (written,
 *            so that the work is not optimised away).
 * The caller times the launch on `stream` (HIP events): cycles per wave
 * instruction per SIMD = time x clock / (waves_per_simd x iters x 16 x chains).
 * Returns 0, 1 for bad arguments, 4 for a device error.
 */
int sdtw_probe_issue(int kind, int chains, int waves_per_simd, int iters, void* out_dev,
                     void* stream);

/*
 * LDS cost of the tile switch's operations: 4 x CUs x waves_per_simd one-wave
 * workgroups spread as above, each running iters blocks of 8 ds_read_b128 +
 * 8 ds_write_b128 on its own 2 KiB of LDS (lane l at 16 l bytes: no bank
 * conflicts) with `lanes` (1..64) lanes active, each block ending with a
 * wait for all of them.  out_dev as for sdtw_probe_issue.  Cycles per LDS
 * instruction per CU = time x clock / (4 x waves_per_simd x iters x 16).
 * Returns 0, 1 for bad arguments, 4 for a device error.
 */
int sdtw_probe_lds(int lanes, int waves_per_simd, int iters, void* out_dev, void* stream);

/*
 * Workgroup placement of a launch of `blocks` workgroups of `threads` threads
 * (a multiple of 64, at most 1024) with `lds_bytes` of dynamic LDS, each wave
 * holding `vgprs` vector registers (0, 150 or 230: those of the alignment
 * kernels whose placement it stands for): wave 0 of each workgroup takes a
 * ticket from the counter out_dev[0] (zero it first), as the persistent
 * alignment kernel takes its first read; every wave w of workgroup b writes
 * (ticket, HW_ID, XCC_ID, start and end of its residency in s_memrealtime
 * ticks, 0, 0, 0) at out_dev[8 + 8 (b x waves + w)], sleeping `spin`
 * (<= 100,000) bounded rounds in between so that the workgroups are resident
 * together.  out_dev: 8 + 8 x blocks x waves uint32.  Returns 0, 1 for bad
 * arguments, 4 for a launch error.
 */
int sdtw_probe_placement(int blocks, int threads, int lds_bytes, int vgprs, int spin,
                         void* out_dev, void* stream);

#ifdef __cplusplus
}
#endif
#endif
