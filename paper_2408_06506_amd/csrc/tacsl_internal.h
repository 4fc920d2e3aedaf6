// Internal layouts shared by the plan builder (tacsl_plan.cpp) and the
// kernels (tacsl_kernels.hip).  Not part of the public ABI.
#pragma once
#include <cstdint>
#include <hip/hip_runtime.h>

namespace tacsl {

// Prepared grid ("2 x 2 columns"): one float4 record per node,
// (phi, G_x, G_y, G_z) with G the nodal finite-difference gradient (central
// inside, one-sided on the faces).  Node (i, j, k) is stored at byte
//   (i >> 1) * stride_q + (j >> 1) * stride_y + k * 64 + (j & 1) * 32 + (i & 1) * 16,
//   stride_y = 64 nz,  stride_q = stride_y * ceil(ny / 2),
// so each 2 x 2 column of nodes runs along z in 64-byte slabs and a 128-byte
// line holds a 2 x 2 x 2 brick (for even nz): fewer distinct lines per
// wavefront of taxels than 2 x 4 (x, z) patches.  The z step of a cell is an
// immediate offset (+64).
inline int64_t grid_record_bytes(int64_t nx, int64_t ny, int64_t nz) { return ((nx + 1) / 2) * ((ny + 1) / 2) * nz * 64; }

// Clear-block mask, stored after the records of each prepared grid: one bit
// per block of 2 x 2 x 2 cells (block b spans nodes 2b .. 2b + 2 per axis,
// clamped to the grid), set when every node value of the block is > 0.  A
// trilinear value inside such a block is then >= 0 in FP32 as well (each
// lerp of non-negative values rounds to a non-negative value), so a taxel
// whose cell lies in a set block is out of contact without its corners.  A
// 32-bit word holds 4 x 4 x 2 blocks (bit (bx & 3) + 4 (by & 3) + 16 (bz & 1));
// word (wx, wy, wz) sits at byte 4 ((wx W_y + wy) W_z + wz) of the mask.
struct MaskDims {
  int64_t wx, wy, wz;
};
inline MaskDims mask_dims(int64_t nx, int64_t ny, int64_t nz) {
  return {(nx / 2 + 3) / 4, (ny / 2 + 3) / 4, (nz / 2 + 1) / 2};
}
inline int64_t grid_mask_bytes(int64_t nx, int64_t ny, int64_t nz) {
  const MaskDims m = mask_dims(nx, ny, nz);
  return (4 * m.wx * m.wy * m.wz + 15) / 16 * 16;
}
inline int64_t prepared_grid_bytes(int64_t nx, int64_t ny, int64_t nz) {
  return grid_record_bytes(nx, ny, nz) + grid_mask_bytes(nx, ny, nz);
}

// Static per-pad record, built at plan creation (device, read-only).
struct InstStatic {
  const float4* grid;   // prepared grid of the pad's object (layout above)
  int64_t tmpl_off;     // first taxel of the pad's template within the template rows
  int64_t out_off;      // global taxel index of the pad's first taxel
  int32_t nx, ny, nz;   // grid nodes per axis
  int32_t env;          // environment of the pad
  int32_t count;        // taxels on the pad
  uint32_t grid_bytes;  // bytes of the prepared grid (< 2^32)
  uint32_t stride_y;    // bytes between consecutive y-pairs
  uint32_t stride_q;    // bytes between consecutive x-pairs
  float ox, oy, oz, h;  // node (0,0,0) in the object frame, node spacing
  int32_t gid;          // object grid index
  uint32_t mask_off;    // byte offset of the clear-block mask within the prepared grid
  uint32_t mask_sx;     // mask bytes between consecutive x-words (4 W_y W_z)
  uint32_t mask_sy;     // mask bytes between consecutive y-words (4 W_z)
};

// Per-step per-pad record written by the prologue (FP64 math, FP32 store).
//   grid coordinates of a taxel:  u = A x_p + b,  A = R / h  (R = object-from-pad rotation)
//   pad-frame normal:             n = R^T n_o = h A^T n_o
//   pad-frame relative velocity:  x_dot = V + W x x_p
struct InstXf {
  float A[9];
  float b[3];
  float V[3];
  float W[3];
  float prm[4];  // k_n, k_d, k_t, mu
  float h;       // node spacing
  uint32_t ok;   // 0 when the pad's inputs were rejected (then A = 0, b = -1)
  float hc;      // exponent p of the penetration in the normal law (1: linear)
};

// One unit of work: taxels [k0, k0 + count) of pad `inst`.
struct Tile {
  int32_t inst, k0, count;
  int32_t env;  // environment of the pad
};

struct PrologueArgs {
  const float* pad_pose;
  const float* obj_pose;
  const float* pad_twist;
  const float* obj_twist;
  const float* params;
  const float* obj_pose_delta;  // may be null
  const InstStatic* stat;
  InstXf* xf;
  int32_t n_inst;
  uint32_t* status;  // may be null
  int32_t* queue;    // dynamic-schedule counter, reset to 0 here
  float hc;          // normal-law exponent copied into every record
  // spatial order (tuning order 5), else null: per-pad spatial bin, and the
  // pad's tile count added to its bin
  uint32_t* sp_hist;                   // [n_sdf * kSpatialBins] (zero on entry)
  int32_t* sp_bin;                     // [n_inst] bin of each pad
  const int64_t* sp_inst_tile_begin;   // [n_inst + 1]
};

// Spatial execution order, rebuilt on the device every call: pads binned by
// object grid and by the position of their origin in the grid (8 x 8 x 8
// coarse cells in Morton order), each object's tiles in that order cut into
// one contiguous run per XCD and interleaved (slot s runs on XCD s % 8).
constexpr int kSpatialBins = 512;
struct SpatialArgs {
  int32_t n_inst, n_sdf, n_tiles;
  int32_t interleave;              // 1: per-XCD interleave of each object's run; 0: plain spatial order
  uint32_t* hist;                  // [n_sdf * kSpatialBins] tiles per bin, left zeroed
  uint32_t* cursor;                // [n_sdf * kSpatialBins] next free tile position of each bin
  const int32_t* bin;              // [n_inst]
  int32_t* grp_tile_begin;         // [n_sdf + 1]
  const int64_t* inst_tile_begin;  // [n_inst + 1]
  int32_t* order;                  // [n_tiles] out: slot -> tile id
};

// State inputs of the per-pad record when the forward kernel computes it
// itself (fused mode: no prologue launch; orders 0-4, static or persistent
// schedules, per-taxel fields without the observation).
struct FusedIn {
  const float* pad_pose;
  const float* obj_pose;
  const float* pad_twist;
  const float* obj_twist;
  const float* params;
  const float* obj_pose_delta;  // may be null
  uint32_t* status;             // may be null
  float hc;
};

struct FwdArgs {
  const Tile* tiles;
  const int32_t* order;  // execution slot -> tile id
  int32_t n_tiles;
  int32_t dynamic;       // 1: persistent dynamic queue
  int32_t* queue;
  const InstStatic* stat;
  const InstXf* xf;
  const float* tmpl;     // [3][tmpl_T]
  int64_t tmpl_T;
  float* depth;          // [T]
  float* normal;         // [3][T]
  float* fn;             // [3][T]
  float* ft;             // [3][T]
  int64_t T;
  float* partial;        // [n_tiles][6] wrench partials (the wrench itself when tiles == pads)
  int32_t mode;          // 1: per-taxel fields; 2: observation pooling; 3: both
  int32_t nonlinear;     // 1: nonlinear normal law (exponent != 1)
  const int32_t* obs_bin;  // [tmpl_T] bin of each template taxel (-1: none), observation modes
  int32_t obs_n;           // bins per pad
  float* obs_partial;      // [n_tiles][obs_n][3] pooled channel sums
  int32_t fused;           // 1: each tile's workgroup computes its pad's record from `fin` (mode 1 only)
  FusedIn fin;
};

// Observation epilogue: per pad and bin, channels (|f_n|, f_t,x, f_t,y)
// averaged over the bin's taxels, divided by scale, clipped to +-clip.
struct ObsReduceArgs {
  const int64_t* inst_tile_begin;  // [n_inst+1]
  const float* partial;            // [n_tiles][obs_n][3]
  const int32_t* inst_tmpl;        // [n_inst]
  const float* icnt;               // [n_tmpl][obs_n] 1 / taxels in the bin (0 for an empty bin)
  float scale[3];                  // per channel, > 0
  float clip;                      // <= 0: no clipping
  int32_t obs_n;
  int32_t n_inst;
  float* obs;                      // [n_inst][obs_n][3]
};

struct WrenchReduceArgs {
  const int64_t* inst_tile_begin;  // [n_inst+1]
  const float* partial;
  float* wrench;
  int32_t n_inst;
};

constexpr int kBwdAcc = 19;  // P1[3] P2[3] N1[3] U1[3] U2[3] (k_n k_d k_t mu)

struct BwdArgs {
  const Tile* tiles;
  const int32_t* order;
  int32_t n_tiles;
  int32_t dynamic;
  int32_t* queue;
  const InstStatic* stat;
  const InstXf* xf;
  const float* tmpl;
  int64_t tmpl_T;
  const float* w_fn;  // [3][T]
  const float* w_ft;  // [3][T]
  int64_t T;
  double* partial;    // [n_tiles][kBwdAcc]
  int32_t nonlinear;  // 1: nonlinear normal law (exponent != 1)
};

struct GradReduceArgs {
  const int32_t* env_inst_begin;   // [n_env+1]
  const int32_t* env_inst;         // pads of each environment, ascending
  const int64_t* inst_tile_begin;  // [n_inst+1]
  const double* partial;           // [n_tiles][kBwdAcc]
  const InstStatic* stat;
  const float* pad_pose;
  const float* obj_pose;
  const float* obj_twist;
  const float* obj_pose_delta;     // may be null
  float* g_obj_pose;               // [n_env][6]
  float* g_obj_twist;              // [n_env][6]
  float* g_params;                 // [n_env][4]
  int32_t n_env;
};

// Node values only, for the depth march ("x-quad columns"): node (i, j, k)
// at byte (i >> 2) * stride_q + j * stride_y + 16 k + 4 (i & 3),
// stride_y = 16 nz, stride_q = stride_y ny, so a 128-byte line holds 4 x-nodes
// by 8 z-nodes at one y (four times the nodes of a line of (phi, G) records).
inline int64_t phi_quad_bytes(int64_t nx, int64_t ny, int64_t nz) { return ((nx + 3) / 4) * ny * nz * 16; }
// Local slope bounds for the sphere steps: per block of 8 x 8 x 8 cells, the
// largest |phi(node + e_k) - phi(node)| along each axis k over the k-edges of
// the cells of the block and of its 26 neighbours (float4: x, y, z, unused).
// Inside a cell each partial derivative of the trilinear field (per grid step)
// interpolates the cell's edge differences with non-negative weights, so it is
// bounded by that maximum anywhere within 8 cells of the block.
constexpr int kSlopeBlock = 8;
inline int64_t slope_blocks(int64_t n) { return (n - 2) / kSlopeBlock + 1; }
struct DepthGrid {
  const float* phi;
  const float4* slope;  // [sbx][sby][sbz]
  uint32_t bytes;
  uint32_t stride_y, stride_q;
  int32_t sby, sbz;
  int32_t pad_;
};

// Tactile depth image: per pad, pixels in 8 x 8 blocks (one wavefront each).
struct DepthArgs {
  const InstStatic* stat;
  const InstXf* xf;
  const DepthGrid* grids;  // [n_sdf] node values per object grid
  const int32_t* pad_order;  // [n_inst] pads in the order their workgroups are dispatched
  int32_t n_inst;
  int32_t rows, cols, ortho;
  float x0, y0, dx, dy;  // pixel grid on the pad plane
  float cam_dist, gel;
  int32_t blocks_x;        // 8 x 8 blocks per image row of blocks
  int32_t blocks_per_pad;
  int32_t wg_per_pad;      // workgroups per pad (set by the launcher)
  float* image;            // [n_inst][rows][cols]
  uint32_t* status;        // may be null
};

// Static device scratch of the allocation-free forward entry point (bytes
// per GPU) and the largest device index it serves.
constexpr int64_t kScratchBytes = int64_t(16) << 20;
constexpr int kMaxScratchDevices = 64;
// Device address of the scratch array on `device`, which must be the current
// device; resolved with hipGetSymbolAddress on the first call per device.
hipError_t scratch_address(int device, void** out);
hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t stream);
hipError_t launch_pose_step(const float* pose0, const float* twist, double t, int32_t n_env, float* pose,
                            hipStream_t stream);
hipError_t launch_spatial_order(const SpatialArgs& a, hipStream_t stream);
hipError_t launch_phi_quad(const float4* grid, int nx, int ny, int nz, float* out, hipStream_t stream);
hipError_t launch_block_slopes(const float* phi4, int nx, int ny, int nz, float4* raw, float4* out, hipStream_t stream);
hipError_t launch_depth_image(const DepthArgs& a, hipStream_t stream);
hipError_t launch_clear_mask(const float* phi, uint32_t* mask, int nx, int ny, int nz, hipStream_t stream);
hipError_t launch_prepare_grid(const float* phi, float4* out, int nx, int ny, int nz, float h,
                               uint32_t* bad_count, hipStream_t stream);
hipError_t launch_prologue(const PrologueArgs& a, hipStream_t stream);
hipError_t launch_forward(const FwdArgs& a, int block, int grid, hipStream_t stream);
hipError_t launch_wrench_reduce(const WrenchReduceArgs& a, hipStream_t stream);
hipError_t launch_obs_reduce(const ObsReduceArgs& a, hipStream_t stream);
hipError_t launch_backward(const BwdArgs& a, int block, int grid, hipStream_t stream);
hipError_t launch_grad_reduce(const GradReduceArgs& a, hipStream_t stream);

}  // namespace tacsl
