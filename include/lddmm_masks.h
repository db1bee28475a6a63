/*
 * Mask generation (Methods, Mask Generation) and the surface metrics of the
 * evaluation (Methods, Evaluation) of the masked LDDMM library, on the GPU.
 *
 * Conventions (all calls):
 *  - Grids are lddmm_grid (x fastest, each axis in [1, LDDMM_MAX_DIM]) with an
 *    isotropic voxel size `spacing` > 0; radii and distances are in the same
 *    physical unit.
 *  - A mask is float32 on the grid; a voxel is in the mask when its value is > 0.
 *    Output masks hold 0 or 1.
 *  - A ball of radius r is the set of integer offsets o with
 *    (spacing |o|)^2 <= r^2, decided in FP64 as |o|^2 <= (r / spacing)^2.
 *  - Voxels outside the grid are background for erosion and dilation.
 *  - Device pointers, asynchronous on `stream`; the workspace is device memory of
 *    lddmm_masks_workspace_size bytes, owned by the caller, no state kept
 *    between calls.  The y pass of lddmm_surface_distance (its dominant
 *    kernel) is timed under LDDMM_PROF_OTHER.
 *  - Returns LDDMM_OK, LDDMM_EINVAL (null pointer, bad grid, bad op, radius
 *    negative or not below (LDDMM_MORPH_MAX_RADIUS_VOXELS + 1) voxels,
 *    workspace too small; nothing launched) or LDDMM_EHIP.
 */
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "lddmm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LDDMM_MORPH_ERODE  0   /* keep x when every voxel of x + ball is in the mask */
#define LDDMM_MORPH_DILATE 1   /* keep x when some voxel of x + ball is in the mask */
#define LDDMM_MORPH_OPEN   2   /* erode, then dilate (removes grains smaller than the ball) */
#define LDDMM_MORPH_CLOSE  3   /* dilate, then erode (fills holes smaller than the ball) */
#define LDDMM_MORPH_MAX_RADIUS_VOXELS 31

/* Bytes of device workspace every call below needs on `grid` (0 if invalid). */
size_t lddmm_masks_workspace_size(const lddmm_grid *grid);

/* Template mask from annotations (Methods, Mask Generation): the union of all
 * foreground labels, mask = 1[label != 0].  labels: int32 [N]; mask: float32 [N]. */
int lddmm_label_mask(const lddmm_grid *grid, const int32_t *labels, float *mask, void *stream);

/* One binary morphology operation with a ball of physical radius `radius`:
 * out = op(mask).  mask, out: float32 [N] (may alias). */
int lddmm_morphology(const lddmm_grid *grid, const float *mask, int32_t op, double radius,
                     float *out, void *workspace, size_t workspace_bytes, void *stream);

/* Target mask (Methods, Mask Generation): threshold the image (1[I > tau]),
 * open with a ball of radius open_radius (50 um in the paper), then close with a
 * ball of radius close_radius (125 um).  image, mask: float32 [N]. */
int lddmm_target_mask(const lddmm_grid *grid, const float *image, float tau, double open_radius,
                      double close_radius, float *mask, void *workspace, size_t workspace_bytes,
                      void *stream);

/*
 * Surface distances (Methods, Evaluation) between two masks on one grid, e.g.
 * the deformed template mask M0 o phi^-1 and the target mask M1.  The surface
 * of a mask is the set of its voxels with at least one of the six face
 * neighbours outside the mask or the grid.  For every voxel of either surface,
 * its distance to the nearest voxel of the other surface is spacing sqrt(k),
 * k the (integer) squared index distance, computed exactly.
 * out (device, 4 doubles): [0] the Hausdorff distance d_H (largest of those
 * distances), [1] the median d_M of all of them from both surfaces (the mean of
 * the two middle values when their count is even), [2] and [3] the number of
 * surface voxels of mask_a and mask_b.  Either surface empty: [0], [1] = NaN.
 */
int lddmm_surface_distance(const lddmm_grid *grid, const float *mask_a, const float *mask_b,
                           double *out, void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif
