// Launch interface of the renderers (macro-cell kernels and the persistent
// sample-streaming marcher), kept apart from the query and training kernels.
#pragma once

#include "kernels.hpp"

namespace ngvol {

struct RenderArgs {
  float cam[12];
  const float* lut;
  int32_t width, height;
  float dt;
  uint32_t seed;
  float* rgba;
  uint32_t* n_geo;
  uint32_t* n_used;
  unsigned long long* counters;  // [4] in the workspace or caller's struct
  unsigned int* queue;           // ray queue head
  McGeom mc;                     // mc.mu set: empty-space skipping, or adaptive marching
  int32_t adaptive;              // with mc.mu: adaptive steps (Section 5.3) instead of skipping only
  float step_max;                // largest step in grid steps (s2)
  int32_t step_exp;              // exponent p of the step formula
  int32_t mode;                  // NGVOL_RENDER_RM, _RM_SHADOW or _PT
  float light[3];                // direction towards the light (normalised on the device)
  uint32_t* aux;                 // per pixel, nullable: shadow point index (RM_SHADOW)
  // path tracing
  float radiance[3];             // light radiance E
  float background[3];           // radiance B of rays leaving the cube
  float density;                 // extinction scale
  int32_t spp, rr_depth, max_depth;
};
hipError_t launch_mc_reset(const McGeom& g, hipStream_t st);
hipError_t launch_mc_update(const McGeom& g, const float* xyz, const float* values, int64_t n, hipStream_t st);
hipError_t launch_mc_opacity(const McGeom& g, const float* lut, hipStream_t st);
size_t render_lds_bytes(const ngvol_plan* plan, int waves);
hipError_t launch_render(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const RenderArgs& ra,
                         hipStream_t st);
template <int P, int W>
hipError_t launch_render_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const RenderArgs& ra,
                           hipStream_t st);
size_t render_pt_lds_bytes(const ngvol_plan* plan, int waves);
template <int P, int W>
hipError_t launch_render_pt_p(const ngvol_plan* plan, TablePtrs tp, const float* mlp, const RenderArgs& ra,
                              hipStream_t st);

}  // namespace ngvol
