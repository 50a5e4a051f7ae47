// The FP32-flux kernels of the batch whose tile bodies run in a persistent
// loop: face (Sec. 3.3 Steps 2-4), Step 1 line and 1-D stage kernels, over
// the tiles of every job as cgks_batch.hip describes.  They are a unit of
// their own because they are compiled without machine loop-invariant code
// motion: inside the item loop it lifts constants out of the loop, the FP64
// ones of the flux's exponentials into vector registers and the stencil
// weights into scalar ones, which then spill (into scratch, or scalars into
// vector lanes); left in the loop body they are rebuilt per tile from
// immediates.  With that the face kernels of stage 2 fit 168 registers
// (three waves per SIMD, kBatchWaves), the 1-D stage 128 (four), and the
// line kernels keep their scalars.  Each face kernel gets a persistent grid
// sized by its own resident blocks per CU.
#define CGKS_UNIT batched_f32
#include "cgks_internal.hpp"

#include <algorithm>

#include "cgks_batch.hpp"

namespace {

// resident blocks per CU of each kernel: [dir][stage - 1][m - 2][tile shape],
// filled when a batch is created (the same for every batch of a process on
// one device type; concurrent creations write the same values)
int g_occ[2][2][3][kFaceTiles];

template <int DIR, int STAGE, int M, int V>
cgks_status prepare1() {
  const void* f = (const void*)kb_face<DIR, STAGE, float, M, V>;
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kb_face_lds<DIR, STAGE, float, M, V>());
  if (e != hipSuccess) return fail(CGKS_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  return check_private(f, 0, "batched face kernel");
}

template <int DIR, int STAGE, int M, int V>
hipError_t occupancy1() {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&g_occ[DIR][STAGE - 1][M - 2][V], kb_face<DIR, STAGE, float, M, V>,
                                                      256, kb_face_lds<DIR, STAGE, float, M, V>());
}

template <int DIR, int STAGE, int M, int V>
void launch1(int ncu, int mult, hipStream_t st, const BTab* t, int r) {
  int g = ncu * std::max(1, g_occ[DIR][STAGE - 1][M - 2][V]) * mult;
  g = (g + 7) & ~7;   // a multiple of 8 (one share per XCD)
  constexpr size_t lds = kb_face_lds<DIR, STAGE, float, M, V>();
  hipLaunchKernelGGL((kb_face<DIR, STAGE, float, M, V>), dim3(g), dim3(256), lds, st, t, r);
}

// the three orders of one direction, stage and tile shape
template <int DIR, int STAGE, int V>
cgks_status prepare_m() {
  cgks_status s;
  if ((s = prepare1<DIR, STAGE, 2, V>()) != CGKS_OK) return s;
  if ((s = prepare1<DIR, STAGE, 3, V>()) != CGKS_OK) return s;
  return prepare1<DIR, STAGE, 4, V>();
}

template <int DIR, int STAGE, int V>
hipError_t occupancy_m() {
  hipError_t e;
  if ((e = occupancy1<DIR, STAGE, 2, V>())) return e;
  if ((e = occupancy1<DIR, STAGE, 3, V>())) return e;
  return occupancy1<DIR, STAGE, 4, V>();
}

template <int DIR, int STAGE, int V>
void launch_m(int ncu, int mult, hipStream_t st, const BTab* t, int r) {
  launch1<DIR, STAGE, 2, V>(ncu, mult, st, t, r);
  launch1<DIR, STAGE, 3, V>(ncu, mult, st, t, r);
  launch1<DIR, STAGE, 4, V>(ncu, mult, st, t, r);
}

template <int V>
cgks_status prepare_v() {
  cgks_status s;
  if ((s = prepare_m<0, 1, V>()) != CGKS_OK) return s;
  if ((s = prepare_m<1, 1, V>()) != CGKS_OK) return s;
  if ((s = prepare_m<0, 2, V>()) != CGKS_OK) return s;
  return prepare_m<1, 2, V>();
}

template <int V>
hipError_t occupancy_v() {
  hipError_t e;
  if ((e = occupancy_m<0, 1, V>())) return e;
  if ((e = occupancy_m<1, 1, V>())) return e;
  if ((e = occupancy_m<0, 2, V>())) return e;
  return occupancy_m<1, 2, V>();
}

template <int V>
void launch_v(int dir, int stage, int ncu, int mult, hipStream_t st, const BTab* t, int r) {
  if (stage == 1) {
    if (dir == 0) launch_m<0, 1, V>(ncu, mult, st, t, r);
    else launch_m<1, 1, V>(ncu, mult, st, t, r);
  } else {
    if (dir == 0) launch_m<0, 2, V>(ncu, mult, st, t, r);
    else launch_m<1, 2, V>(ncu, mult, st, t, r);
  }
}

}  // namespace

namespace cgks_bf32 {

cgks_status prepare() {
  cgks_status s;
  if ((s = prepare_v<0>()) != CGKS_OK) return s;
  if ((s = prepare_v<1>()) != CGKS_OK) return s;
  if ((s = prepare_v<2>()) != CGKS_OK) return s;
  const void* k[] = {(const void*)kb_lines<0, float>, (const void*)kb_lines<1, float>, (const void*)kb_stage1d<1, float>,
                     (const void*)kb_stage1d<2, float>};
  for (const void* f : k)
    if ((s = check_private(f, 0, "batched kernel")) != CGKS_OK) return s;
  return CGKS_OK;
}

hipError_t occupancy(int occ_face[kFaceTiles], int occ_lines[kLineTiles], int* occ_s1d) {
  hipError_t e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_lines[0], kb_lines<0, float>, 256, 0))) return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_lines[1], kb_lines<1, float>, 256, 0))) return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(occ_s1d, kb_stage1d<2, float>, 256, 0))) return e;
  if ((e = occupancy_v<0>())) return e;
  if ((e = occupancy_v<1>())) return e;
  if ((e = occupancy_v<2>())) return e;
  for (int v = 0; v < kFaceTiles; ++v) {
    int m = 1 << 30;
    for (int d = 0; d < 2; ++d)
      for (int s = 0; s < 2; ++s)
        for (int k = 0; k < 3; ++k) m = std::min(m, g_occ[d][s][k][v]);
    occ_face[v] = m;
  }
  return hipSuccess;
}

void launch_faces(int dir, int stage, int v, int ncu, int mult, hipStream_t st, const void* tab, int remap) {
  const BTab* t = (const BTab*)tab;
  switch (v) {
    case 1: launch_v<1>(dir, stage, ncu, mult, st, t, remap); break;
    case 2: launch_v<2>(dir, stage, ncu, mult, st, t, remap); break;
    default: launch_v<0>(dir, stage, ncu, mult, st, t, remap); break;
  }
}

void launch_lines(int lw, int grid, hipStream_t st, const void* tab, int stage, int remap) {
  const BTab* t = (const BTab*)tab;
  if (lw == 1) hipLaunchKernelGGL((kb_lines<1, float>), dim3(grid), dim3(256), 0, st, t, stage, remap);
  else hipLaunchKernelGGL((kb_lines<0, float>), dim3(grid), dim3(256), 0, st, t, stage, remap);
}

void launch_stage1d(int stage, int grid, hipStream_t st, const void* tab, int remap) {
  const BTab* t = (const BTab*)tab;
  if (stage == 1) hipLaunchKernelGGL((kb_stage1d<1, float>), dim3(grid), dim3(256), 0, st, t, remap);
  else hipLaunchKernelGGL((kb_stage1d<2, float>), dim3(grid), dim3(256), 0, st, t, remap);
}

}  // namespace cgks_bf32
