// Batched execution, shared by the translation units of the batched
// kernels: the device job table, the persistent item loop, and the batched
// Step 1 line, 1-D stage and face kernels.  Their FP64 instances are built
// with the rest of the batch (cgks_batch.hip), the FP32 ones in a unit of
// their own (cgks_batch_f32.hip), compiled without machine loop-invariant
// code motion.  Included after cgks_internal.hpp.
#pragma once
namespace {

// Phases of a step, in launch order (2-D; 1-D uses DT, PREP, S1D1, BCS, S1D2).
// The face phases are per order m: each has a kernel compiled for that m
// alone, which keeps its registers within the register file.
enum Phase { PH_DT = 0, PH_PREP, PH_LINES, PH_FX2, PH_FX3, PH_FX4, PH_FY2, PH_FY3, PH_FY4, PH_BCS, PH_S1D, NPH };
constexpr int ph_face(int dir, int m) { return (dir == 0 ? PH_FX2 : PH_FY2) + (m - 2); }

struct BJob {
  Geo g;
  Consts C;
  Bufs B;
  double dt_fixed, cfl, t_end, h;
  double sbc;              // largest |U| + c of the job's prescribed boundary states
  long long max_steps;
  int viscous, M, slot, pad;
  int ax, ay;              // 256-wide segments per row: sigma x-faces, sigma y-faces
  int nsx, nsy;            // PREP items of the sigma x / y parts
  int fnb[2][2];           // face tiles (along normal, along tangential) of x- and y-faces
  int ltx, lty;            // Step 1 tiles along x and y
  int nseg;                // 1-D stage segments
  int ns;                  // ghost-cell items (GhostItems)
};

struct S1Item {
  int job, seg;   // job (table order), item index within the job
};

struct BTab {
  int njobs, cap;
  int total[NPH];
  BJob* jobs;      // [cap], table order
  int* pre;        // [NPH][cap + 1] prefix sums of the items per job
  JobStat* stat;   // [cap], by slot
  // 1-D: the (job, index in the job) of every item of each phase, at
  // imap + ioff[phase] (null in 2-D, whose batches hold few jobs); a 1-D
  // batch has thousands of jobs of a few items each, and a binary search of
  // the prefix sums would cost a dozen dependent loads per item
  S1Item* imap;
  int ioff[NPH];
};

// Largest j in [0, n) with pre[j] <= item (pre[0] = 0, pre[n] = total).
template <class P>
__device__ __forceinline__ int find_job(P pre, int n, int item) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= item) lo = mid;
    else hi = mid;
  }
  return lo;
}

// A job's descriptor, read in place through a pointer of constant type: the
// table does not change while a kernel runs, so its fields are scalar loads
// that the compiler may repeat where they are used, as it does with kernel
// arguments, instead of holding the whole descriptor in registers across a
// tile (through the generic table pointer they would be FLAT loads, which
// count against the LDS counter).  The host pass, which cannot form that
// address space, reads it directly.
__device__ __forceinline__ const BJob& job_ref(const BTab* tab, int j) {
#if defined(__HIP_DEVICE_COMPILE__)
  using cjob = const __attribute__((address_space(4))) BJob*;
  return *(const BJob*)((cjob)tab->jobs + j);
#else
  return tab->jobs[j];
#endif
}

// Persistent loop over the items of a phase.  With remap, blocks that the
// dispatcher places on one XCD (block b runs on XCD b mod 8) take
// consecutive items, so neighbouring tiles of a grid share that XCD's L2.
// CREF: read the job descriptor in place through a constant pointer (the
// default), or copy it (the FP64 face kernels, whose registers are full:
// there the in-place reads cost scratch).
// MAP: the phase may run in a 1-D batch, whose items come from the item map
// when it is present (the 2-D-only kernels leave the branch out: their
// scalar registers are full).
template <bool CREF = true, bool MAP = false, class F>
__device__ __forceinline__ void for_items(const BTab* tab, int ph, int remap, F&& f) {
  const int total = tab->total[ph];
  const int G = gridDim.x;
  int lb = blockIdx.x;
  if (remap) lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);   // G is a multiple of 8
  const int n = tab->njobs;
  const gptr<const int> pre = glb((const int*)tab->pre) + (size_t)ph * (tab->cap + 1);
  const S1Item* imap = MAP ? tab->imap : nullptr;
  for (int item = lb; item < total; item += G) {
    // the job and tile are the same for the whole block: made wave-uniform,
    // the job descriptor comes through scalar loads instead of occupying
    // vector registers.  1-D batches read them from the item map.
    int j, k;
    if (MAP && imap) {
#if defined(__HIP_DEVICE_COMPILE__)
      const S1Item e = glb(imap)[tab->ioff[ph] + item];
#else
      const S1Item e = imap[tab->ioff[ph] + item];
#endif
      j = __builtin_amdgcn_readfirstlane(e.job);
      k = __builtin_amdgcn_readfirstlane(e.seg);
    } else {
      j = __builtin_amdgcn_readfirstlane(find_job(pre, n, item));
      k = __builtin_amdgcn_readfirstlane(item - pre[j]);
    }
#if defined(__HIP_DEVICE_COMPILE__)
    if (CREF) {
      f(job_ref(tab, j), k);
    } else {
      // a copy, read through a pointer of global type: scalar loads
      const BJob J = glb((const BJob*)tab->jobs)[j];
      f(J, k);
    }
#else
    f(tab->jobs[j], k);
#endif
  }
}

// Step 1 line values of the stage input (2-D), one tile of shape LW per item.
template <int LW, typename ST>
__global__ __launch_bounds__(256) void kb_lines(const BTab* tab, int stage, int remap) {
  __shared__ double sm[LinesLds<LW>::total];
  for_items<false>(tab, PH_LINES, remap, [&](const BJob& J, int k) {
    if (!J.B.hdr->active) return;
    const double* Uin = stage == 1 ? J.B.U : J.B.S;
    const int bx = k % J.ltx, by = k / J.ltx;
    switch (J.M) {
      case 2: lines_tile<2, ST, true, LW>(J.g, J.C, Uin, J.B.sxo, J.B.syo, J.B.lvx, J.B.lvy, J.B.hdr, bx, by, sm); break;
      case 3: lines_tile<3, ST, true, LW>(J.g, J.C, Uin, J.B.sxo, J.B.syo, J.B.lvx, J.B.lvy, J.B.hdr, bx, by, sm); break;
      default: lines_tile<4, ST, true, LW>(J.g, J.C, Uin, J.B.sxo, J.B.syo, J.B.lvx, J.B.lvy, J.B.hdr, bx, by, sm); break;
    }
  });
}


// One stage of the 1-D scheme over the segments of every job.
template <int STAGE, typename T>
__global__ __launch_bounds__(256, sizeof(T) == 4 ? 4 : 2) void kb_stage1d(const BTab* tab, int remap) {
  const int total = tab->total[PH_S1D];
  const int G = gridDim.x;
  int lb = blockIdx.x;
  if (remap) lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);   // G is a multiple of 8
  // the item's job and segment (wave-uniform): scalar loads through a
  // pointer of constant type, the map does not change while the kernel runs
  auto item_of = [&](int item, int& j, int& seg) {
#if defined(__HIP_DEVICE_COMPILE__)
    const S1Item e = ((const __attribute__((address_space(4))) S1Item*)tab->imap)[tab->ioff[PH_S1D] + item];
#else
    const S1Item e = tab->imap[tab->ioff[PH_S1D] + item];
#endif
    j = __builtin_amdgcn_readfirstlane(e.job);
    seg = __builtin_amdgcn_readfirstlane(e.seg);
  };
  if constexpr (sizeof(T) == 4) {
    // FP32: inputs copied into LDS by DMA; the descriptor read in place
    // (four waves per SIMD, built without machine loop-invariant code
    // motion)
    __shared__ S1In<T> in;
    __shared__ S1Acc<T> acc;
    __shared__ S1Mid<T, STAGE> mid;
    for (int item = lb; item < total; item += G) {
      int j, seg;
      item_of(item, j, seg);
      const BJob& J = job_ref(tab, j);
      __syncthreads();   // the previous segment is done with the LDS
      s1_issue_in<STAGE, T>(J.g, J.B, seg, &in, tile_tid256());
      s1_landed();
      stage1d_seg_lds<STAGE, T, false, true>(J.g, J.C, J.B, &in, &acc, &mid, seg, J.nseg);
    }
  } else {
    // FP64: inputs through registers; a copy of the descriptor (its scalar
    // registers are full: fields read in place would be reloaded, and waited
    // for, at every use)
    __shared__ double res[256][12];
    __shared__ __align__(16) unsigned char sm[Lds1D<T>::total];
    for (int item = lb; item < total; item += G) {
      int j, seg;
      item_of(item, j, seg);
#if defined(__HIP_DEVICE_COMPILE__)
      const BJob J = glb((const BJob*)tab->jobs)[j];
#else
      const BJob& J = tab->jobs[j];
#endif
      stage1d_seg<STAGE, T, false>(J.g, J.C, J.B, res, sm, seg, J.nseg);
    }
  }
}

// Waves per SIMD of the batched face kernels.  FP32: three at stage 2, whose
// tiles fit 168 registers without scratch inside the persistent loop; two at
// stage 1 (one to five registers over).  FP64: one (the shared layout, as the
// single-grid FP64 kernels).
template <typename T, int DIR, int STAGE, int M>
constexpr int kBatchWaves = sizeof(T) == 8 ? 1 : (STAGE == 1 ? 2 : 3);

// Fused reconstruction + flux + update of one direction and stage over the
// face tiles (shape V) of every job of order m = M.  FP32: the tile body's
// thread index is opaque in each pass of the loop (PERSIST), and the LDS is
// laid out for the kernel's own direction and wave count.
template <int DIR, int STAGE, typename T, int M, int V>
__global__ __launch_bounds__(256, (kBatchWaves<T, DIR, STAGE, M>)) void kb_face(const BTab* tab, int remap) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr bool F32 = sizeof(T) == 4;
  for_items<F32>(tab, ph_face(DIR, M), remap, [&](const BJob& J, int k) {
    const int nbx = J.fnb[DIR][0], nby = J.fnb[DIR][1];
    // neighbours along x first (x-faces: normal-first, y-faces: tangential-first)
    const int bx = DIR == 0 ? k % nbx : k / nby, by = DIR == 0 ? k / nbx : k % nby;
    face2d_tile<DIR, STAGE, M, T, false, 32, F32, V, F32, F32 ? kBatchWaves<T, DIR, STAGE, M> : 0>(J.g, J.C, J.B, smem, bx, by,
                                                                                              nbx, nby);
  });
}

// dynamic LDS of a batched face kernel
template <int DIR, int STAGE, typename T, int M, int V>
constexpr size_t kb_face_lds() {
  return FaceLds<DIR, M, T, V, sizeof(T) == 4 ? kBatchWaves<T, DIR, STAGE, M> : 0>::total;
}

}  // namespace

// The FP32 kernels of the batch that run the tile bodies in a persistent
// loop (cgks_batch_f32.hip): face, Step 1 line and 1-D stage kernels.
//   prepare: their LDS limits and scratch check;
//   occupancy: resident blocks per CU (face kernels: kept per kernel and
//     reported for each tile shape as the fewest over its kernels; line
//     kernels per tile shape; the 1-D stage);
//   launch_faces: one direction and stage, one launch per order, for tile
//     shape v, each a persistent grid of ncu x its resident blocks x mult;
//   launch_lines, launch_stage1d: with the grid the caller sized.
namespace cgks_bf32 {
cgks_status prepare();
hipError_t occupancy(int occ_face[kFaceTiles], int occ_lines[kLineTiles], int* occ_s1d);
void launch_faces(int dir, int stage, int v, int ncu, int mult, hipStream_t st, const void* tab, int remap);
void launch_lines(int lw, int grid, hipStream_t st, const void* tab, int stage, int remap);
void launch_stage1d(int stage, int grid, hipStream_t st, const void* tab, int remap);
}  // namespace cgks_bf32
