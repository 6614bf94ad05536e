/* Phase clock of the directional sweep: a measurement build of the same
 * library (libwenomhd_clock.so, compiled with -DWM_SWEEP_CLOCK; the product
 * library libwenomhd.so neither has the stamps nor exports this call).
 *
 * In the clock build every wave of the sweep kernel (Sect. 2.2 flux
 * evaluation: zone prologue, face state and differences, then the face
 * eigensystem and characteristic WENO) reads the shader clock at its phase
 * boundaries and its lane 0 writes 8 unsigned 64-bit values per wave:
 *   [0] start, [1] zone prologue stored to LDS, [2] after the first barrier,
 *   [3] central flux / face state / differences formed, [4] after the
 *   difference stores and their barriers, [5] eigensystem and WENO done,
 *   [6] flux stores issued, [7] the hardware id of the wave's compute unit.
 * Layout: stamps[(block * 4 + wave) * 8 + q], block the linear id
 * (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x of the launch.
 */
#ifndef WENOMHD_CLOCK_H
#define WENOMHD_CLOCK_H

#include <stddef.h>

#include "wenomhd.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Registers a device buffer of n_stamps unsigned 64-bit values for the sweeps
 * along `axis` (0, 1, 2); stamps = NULL unregisters.  Process-wide (all
 * patches, not thread-safe); a launch whose blocks need more than n_stamps
 * values writes none.  The buffer stays owned by the caller, who keeps it
 * alive while registered.  Returns WM_ERR_ARG for an invalid axis. */
wm_status wm_clock_sweep_buffer(int axis, void* stamps, size_t n_stamps);

#ifdef __cplusplus
}
#endif

#endif /* WENOMHD_CLOCK_H */
