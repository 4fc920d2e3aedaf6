// HIP kernels of the tactile force field for gfx950 (MI355X).
//
// The method is the penalty force field of the TacSL paper, Section III-C:
// query the object's SDF at every tactile point (trilinear), take the
// contact normal from finite-difference SDF gradients, and apply
//   f_n = (-k_n + k_d d_dot) d n,   f_t = -(v_t/|v_t|) min(k_t |v_t|, mu |f_n|),
// with d_dot = n . x_dot (chain rule of Section III-C).
//
// Kernels
//   k_prepare_grid  once per plan: node value + nodal finite-difference
//                   gradient as one float4 record per node, in 2 x 2 columns.
//   k_prologue      per pad, FP64: relative pose and twist, folded into an
//                   affine map taxel -> grid coordinates (FP32 record).
//   k_force_fwd     per tile of taxels: the whole per-taxel path, SoA stores,
//                   per-tile wrench partial (fixed-order reduction).
//   k_wrench_reduce pads split over several tiles: sum partials in tile order.
//   k_force_bwd     hand-written adjoint with recomputation of the forward.
//   k_grad_reduce   per environment, FP64: partials -> world-frame gradients.
//
// Design notes (gfx950): wave64, one taxel per lane per iteration; template
// positions and outputs are SoA so every load/store instruction moves 256
// contiguous bytes per wave; each of the eight corners of a taxel's cell is
// one 16-byte record (value and gradient), so a taxel costs eight gather
// instructions (fewer, wider gathers are what the vector L1 handles best);
// records are laid out so a 128-byte line holds a 2 x 2 x 2 brick of nodes
// (a wavefront's gathers touch a third fewer lines than with x-fastest rows)
// and are fetched through a
// bounds-checked buffer resource (an out-of-range offset reads zeros instead
// of faulting); per-pad constants live in scalar registers; reductions are
// fixed-order (deterministic, no float atomics).
#include <hip/hip_runtime.h>

#include <mutex>

#include "tacsl.h"
#include "tacsl_device.h"
#include "tacsl_internal.h"

namespace tacsl {
namespace {

// Clear-block mask (layout in tacsl_internal.h): one thread per 32-bit word.
__global__ __launch_bounds__(256) void k_clear_mask(const float* __restrict__ phi, uint32_t* __restrict__ mask,
                                                    int nx, int ny, int nz, int wx, int wy, int wz) {
  const int64_t n = (int64_t)wx * wy * wz;
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n) return;
  const int iz = (int)(w % wz), iy = (int)((w / wz) % wy), ix = (int)(w / ((int64_t)wz * wy));
  uint32_t bits = 0u;
  for (int b = 0; b < 32; ++b) {
    const int bx = 4 * ix + (b & 3), by = 4 * iy + ((b >> 2) & 3), bz = 2 * iz + (b >> 4);
    if (2 * bx > nx - 2 || 2 * by > ny - 2 || 2 * bz > nz - 2) continue;  // no cell starts in this block
    bool clear = true;
    for (int k = 2 * bz; clear && k <= min(2 * bz + 2, nz - 1); ++k)
      for (int j = 2 * by; clear && j <= min(2 * by + 2, ny - 1); ++j)
        for (int i = 2 * bx; i <= min(2 * bx + 2, nx - 1); ++i)
          if (!(phi[((int64_t)k * ny + j) * nx + i] > 0.f)) {
            clear = false;
            break;
          }
    if (clear) bits |= 1u << b;
  }
  mask[w] = bits;
}

// ---------------------------------------------------------------------------
// SDF preparation: (phi, G) per node, G = nodal finite differences (central
// inside, one-sided on the faces), stored in the 2 x 2 column layout.
// Counts non-finite node values.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prepare_grid(const float* __restrict__ phi, float4* __restrict__ out,
                                                      int nx, int ny, int nz, float h,
                                                      uint32_t* __restrict__ bad) {
  const int64_t n = (int64_t)nx * ny * nz;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % nx);
    const int j = (int)((idx / nx) % ny);
    const int k = (int)(idx / ((int64_t)nx * ny));
    const float p = phi[idx];
    const int il = i > 0 ? i - 1 : 0, ih = i < nx - 1 ? i + 1 : nx - 1;
    const int jl = j > 0 ? j - 1 : 0, jh = j < ny - 1 ? j + 1 : ny - 1;
    const int kl = k > 0 ? k - 1 : 0, kh = k < nz - 1 ? k + 1 : nz - 1;
    const int64_t row = ((int64_t)k * ny + j) * nx;
    const float gx = (phi[row + ih] - phi[row + il]) / ((float)(ih - il) * h);
    const float gy = (phi[((int64_t)k * ny + jh) * nx + i] - phi[((int64_t)k * ny + jl) * nx + i]) /
                     ((float)(jh - jl) * h);
    const float gz = (phi[((int64_t)kh * ny + j) * nx + i] - phi[((int64_t)kl * ny + j) * nx + i]) /
                     ((float)(kh - kl) * h);
    if (!isfinite(p)) atomicAdd(bad, 1u);
    const int64_t rec = ((int64_t)(i >> 1) * ((ny + 1) / 2) + (j >> 1)) * nz * 4 + (int64_t)k * 4 + (j & 1) * 2 + (i & 1);
    out[rec] = make_float4(p, gx, gy, gz);
  }
}

// ---------------------------------------------------------------------------
// Prologue (FP64): per pad, object-from-pad rotation R, the affine map to grid
// coordinates u = A x + b (A = R/h, b = (R_o^T (t_p - t_o) - origin)/h) and
// the pad-frame relative velocity field x_dot = V + W x x_p with
//   V = R_p^T [(v_p - v_o) - w_o x (t_p - t_o)],  W = R_p^T (w_p - w_o).
// ---------------------------------------------------------------------------
__device__ bool quat_to_R(const float* q, double R[9], uint32_t& bits) {
#pragma clang fp contract(off)
  double w = q[0], x = q[1], y = q[2], z = q[3];
  double n2 = w * w + x * x + y * y + z * z;
  if (!(n2 > 0.0)) {
    bits |= 0x2u;
    return false;
  }
  double inv = 1.0 / sqrt(n2);
  w *= inv; x *= inv; y *= inv; z *= inv;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
  return true;
}

// Rotation matrix of the rotation vector p (Rodrigues; series for tiny angles).
__device__ void rotvec_to_R(const double p[3], double R[9]) {
#pragma clang fp contract(off)
  const double t2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  double a, b;
  if (t2 < 1e-12) {
    a = 1.0 - t2 / 6.0;
    b = 0.5 - t2 / 24.0;
  } else {
    const double t = sqrt(t2);
    a = sin(t) / t;
    b = (1.0 - cos(t)) / t2;
  }
  const double K[9] = {0, -p[2], p[1], p[2], 0, -p[0], -p[1], p[0], 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double k2 = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
      R[3 * i + j] = (i == j ? 1.0 : 0.0) + a * K[3 * i + j] + b * k2;
    }
}

__device__ bool all_finite(const float* p, int n) {
  bool ok = true;
  for (int i = 0; i < n; ++i) ok &= isfinite(p[i]);
  return ok;
}

// Object world pose after the optional perturbation (FP64).
__device__ bool object_pose(const float* obj_pose, const float* delta, double Ro[9], double to[3],
                            uint32_t& bits) {
#pragma clang fp contract(off)
  if (!quat_to_R(obj_pose, Ro, bits)) return false;
  for (int a = 0; a < 3; ++a) to[a] = obj_pose[4 + a];
  if (delta) {
    const double th[3] = {delta[3], delta[4], delta[5]};
    double E[9], M[9];
    rotvec_to_R(th, E);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) M[3 * i + j] = E[3 * i] * Ro[j] + E[3 * i + 1] * Ro[3 + j] + E[3 * i + 2] * Ro[6 + j];
    for (int i = 0; i < 9; ++i) Ro[i] = M[i];
    for (int a = 0; a < 3; ++a) to[a] += delta[a];
  }
  return true;
}

// The record of pad i (and the status bits its inputs raise).  No FP
// contraction here or in the helpers above: the record has the same bits in
// k_prologue and in the fused forward kernel, whatever the surrounding code.
__device__ __forceinline__ void pad_record(const float* pad_pose, const float* obj_pose, const float* pad_twist,
                                           const float* obj_twist, const float* params, const float* obj_pose_delta,
                                           const InstStatic& st, int64_t i, int e, float hc, InstXf& x,
                                           uint32_t& bits) {
#pragma clang fp contract(off)
  const float* pp = pad_pose + 7 * i;
  const float* op = obj_pose + 7 * (int64_t)e;
  const float* pt = pad_twist + 6 * i;
  const float* ot = obj_twist + 6 * (int64_t)e;
  const float* pr = params + 4 * (int64_t)e;
  const float* dl = obj_pose_delta ? obj_pose_delta + 6 * (int64_t)e : nullptr;
  bool ok = all_finite(pp, 7) && all_finite(op, 7) && all_finite(pt, 6) && all_finite(ot, 6) &&
            all_finite(pr, 4) && (dl == nullptr || all_finite(dl, 6));
  if (!ok) bits |= 0x1u;
  double Rp[9], Ro[9], to[3];
  if (ok) ok = quat_to_R(pp, Rp, bits);
  if (ok) ok = object_pose(op, dl, Ro, to, bits);
  if (ok) {
    const double tp[3] = {pp[4], pp[5], pp[6]};
    const double d[3] = {tp[0] - to[0], tp[1] - to[1], tp[2] - to[2]};
    double R[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) R[3 * r + c] = Ro[r] * Rp[c] + Ro[3 + r] * Rp[3 + c] + Ro[6 + r] * Rp[6 + c];
    const double top[3] = {Ro[0] * d[0] + Ro[3] * d[1] + Ro[6] * d[2], Ro[1] * d[0] + Ro[4] * d[1] + Ro[7] * d[2],
                           Ro[2] * d[0] + Ro[5] * d[1] + Ro[8] * d[2]};
    const double h = st.h;
    const double org[3] = {st.ox, st.oy, st.oz};
    for (int k = 0; k < 9; ++k) x.A[k] = (float)(R[k] / h);
    x.h = st.h;
    for (int r = 0; r < 3; ++r) x.b[r] = (float)((top[r] - org[r]) / h);
    const double wo[3] = {ot[3], ot[4], ot[5]};
    const double dv[3] = {pt[0] - ot[0] - (wo[1] * d[2] - wo[2] * d[1]), pt[1] - ot[1] - (wo[2] * d[0] - wo[0] * d[2]),
                          pt[2] - ot[2] - (wo[0] * d[1] - wo[1] * d[0])};
    const double dw[3] = {pt[3] - ot[3], pt[4] - ot[4], pt[5] - ot[5]};
    for (int r = 0; r < 3; ++r) {
      x.V[r] = (float)(Rp[r] * dv[0] + Rp[3 + r] * dv[1] + Rp[6 + r] * dv[2]);
      x.W[r] = (float)(Rp[r] * dw[0] + Rp[3 + r] * dw[1] + Rp[6 + r] * dw[2]);
    }
    for (int k = 0; k < 4; ++k) x.prm[k] = pr[k];
    x.ok = 1;
  } else {
    for (int k = 0; k < 9; ++k) x.A[k] = 0.f;
    x.h = 0.f;
    for (int k = 0; k < 3; ++k) { x.b[k] = -1.f; x.V[k] = 0.f; x.W[k] = 0.f; }
    for (int k = 0; k < 4; ++k) x.prm[k] = 0.f;
    x.ok = 0;
  }
  x.hc = hc;
}

__global__ __launch_bounds__(64) void k_prologue(PrologueArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && a.queue) *a.queue = 0;
  if (i >= a.n_inst) return;
  const InstStatic st = a.stat[i];
  uint32_t bits = 0;
  InstXf x;
  pad_record(a.pad_pose, a.obj_pose, a.pad_twist, a.obj_twist, a.params, a.obj_pose_delta, st, i, st.env, a.hc, x,
             bits);
  a.xf[i] = x;
  if (bits && a.status) atomicOr(a.status, bits);
  if (a.sp_hist) {
    // coarse cell of the pad origin (u = b) in its grid, 8 per axis, Morton order
    const int n3[3] = {st.nx, st.ny, st.nz};
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float cf = x.b[k] * 8.f / (float)(n3[k] - 1);
      const uint32_t cb = (uint32_t)min(max((int)floorf(cf), 0), 7);
#pragma unroll
      for (int bit = 0; bit < 3; ++bit) m |= ((cb >> bit) & 1u) << (3 * bit + k);
    }
    const int bin = st.gid * kSpatialBins + (int)m;
    a.sp_bin[i] = bin;
    atomicAdd(a.sp_hist + bin, (uint32_t)(a.sp_inst_tile_begin[i + 1] - a.sp_inst_tile_begin[i]));
  }
}

// Exclusive prefix of the bins' tile counts, in rounds of 1024 (one
// workgroup): the next free position of each bin, the first tile of each
// object grid, and the counts cleared for the next call.
__global__ __launch_bounds__(1024) void k_sp_scan(const SpatialArgs a) {
  __shared__ uint32_t lds[1024];
  const int n = a.n_sdf * kSpatialBins;
  const int t = threadIdx.x;
  uint32_t carry = 0;
  for (int base = 0; base < n; base += 1024) {
    const int k = base + t;
    const uint32_t v = k < n ? a.hist[k] : 0u;
    lds[t] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const uint32_t add = t >= o ? lds[t - o] : 0u;
      __syncthreads();
      lds[t] += add;
      __syncthreads();
    }
    const uint32_t excl = carry + lds[t] - v;
    if (k < n) {
      a.cursor[k] = excl;
      a.hist[k] = 0u;
      if (k % kSpatialBins == 0) a.grp_tile_begin[k / kSpatialBins] = (int32_t)excl;
    }
    carry += lds[1023];
    __syncthreads();
  }
  if (t == 0) a.grp_tile_begin[a.n_sdf] = (int32_t)carry;
}

// Each pad takes the next run of its bin's tile positions (any order within
// a bin) and writes its tiles into the slots of the per-XCD interleave.
__global__ __launch_bounds__(256) void k_sp_place(const SpatialArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n_inst) return;
  const int bin = a.bin[i];
  const int64_t t0 = a.inst_tile_begin[i];
  const int cnt = (int)(a.inst_tile_begin[i + 1] - t0);
  const int pos = (int)atomicAdd(a.cursor + bin, (uint32_t)cnt);
  const int g = bin / kSpatialBins;
  const int A = a.grp_tile_begin[g], n = a.grp_tile_begin[g + 1] - A;
  const int q = n >> 3, r = n & 7;
  for (int k = 0; k < cnt; ++k) {
    const int jr = pos + k - A;  // rank in the object's spatially ordered tiles
    int seg, off;
    if (jr < r * (q + 1)) {
      seg = jr / (q + 1);
      off = jr - seg * (q + 1);
    } else {
      const int j2 = jr - r * (q + 1);
      seg = r + j2 / q;
      off = j2 - (seg - r) * q;
    }
    const int slot = a.interleave ? A + (off < q ? off * 8 + seg : 8 * q + seg) : A + jr;
    if (slot >= 0 && slot < a.n_tiles) a.order[slot] = (int32_t)(t0 + k);  // always true when counts agree
  }
}


// ---------------------------------------------------------------------------
// Per-taxel forward (shared by the forward and the adjoint kernels).
// ---------------------------------------------------------------------------
struct TaxelFwd {
  bool contact;  // inside the node box and phi < 0
  bool force;    // contact and |g|^2 >= 1e-12
  float ux, uy, uz;
  float tx, ty, tz;
  float4 c[8];   // corner records (phi, G), index dx + 2 dy + 4 dz
  float phi;
  float gx, gy, gz, r;
  float nox, noy, noz;
  float n[3];
  float v[3];
  float dd, s;
  float w, dw;  // penetration term of the normal law and its derivative in phi
  float vt[3];
  float vtn, cap;
  bool stick;
  float fn[3], ft[3];
};


// NL: the nonlinear normal law (penetration exponent x.hc != 1), a template
// argument so that the linear law carries no code for it.
template <bool NL>
__device__ __forceinline__ void taxel_forward(const InstXf& x, const InstStatic& st, __amdgpu_buffer_rsrc_t rs,
                                              float px, float py, float pz, TaxelFwd& f) {
  f.contact = false;
  f.force = false;
  f.ux = fmaf(x.A[0], px, fmaf(x.A[1], py, fmaf(x.A[2], pz, x.b[0])));
  f.uy = fmaf(x.A[3], px, fmaf(x.A[4], py, fmaf(x.A[5], pz, x.b[1])));
  f.uz = fmaf(x.A[6], px, fmaf(x.A[7], py, fmaf(x.A[8], pz, x.b[2])));
  const bool in = (f.ux >= 0.f) && (f.ux <= (float)(st.nx - 1)) && (f.uy >= 0.f) &&
                  (f.uy <= (float)(st.ny - 1)) && (f.uz >= 0.f) && (f.uz <= (float)(st.nz - 1));
  if (!in) return;
  const int cx = min((int)floorf(f.ux), st.nx - 2);
  const int cy = min((int)floorf(f.uy), st.ny - 2);
  const int cz = min((int)floorf(f.uz), st.nz - 2);
  f.tx = f.ux - (float)cx;
  f.ty = f.uy - (float)cy;
  f.tz = f.uz - (float)cz;
  {
    // cells in a clear block are out of contact: skip their eight gathers
    const uint32_t bx = (uint32_t)cx >> 1, by = (uint32_t)cy >> 1, bz = (uint32_t)cz >> 1;
    const uint32_t mo = st.mask_off + __umul24(bx >> 2, st.mask_sx) + __umul24(by >> 2, st.mask_sy) + (bz >> 1) * 4u;
    const uint32_t word = __builtin_amdgcn_raw_buffer_load_b32(rs, mo, 0u, 0);
    if ((word >> ((bx & 3u) | ((by & 3u) << 2) | ((bz & 1u) << 4))) & 1u) return;
  }
  // per-lane offsets of the four (x, y) corner columns; the z step is an
  // immediate offset.  Plan creation keeps stride_q = 64 ceil(ny / 2) nz below
  // 2^24 (and so stride_y and the cell indices), so the products fit the
  // full-rate 24-bit multiplier.
  const uint32_t x0 = (uint32_t)cx, x1 = x0 + 1u, y0 = (uint32_t)cy, y1 = y0 + 1u;
  const uint32_t z = (uint32_t)cz * 64u;
  const uint32_t ox0 = __umul24(x0 >> 1, st.stride_q) + (x0 & 1u) * 16u + z;
  const uint32_t ox1 = __umul24(x1 >> 1, st.stride_q) + (x1 & 1u) * 16u + z;
  const uint32_t oy0 = __umul24(y0 >> 1, st.stride_y) + (y0 & 1u) * 32u;
  const uint32_t oy1 = __umul24(y1 >> 1, st.stride_y) + (y1 & 1u) * 32u;
  const uint32_t o00 = ox0 + oy0, o10 = ox1 + oy0, o01 = ox0 + oy1, o11 = ox1 + oy1;
  f.c[0] = load_node(rs, o00, 0u);
  f.c[1] = load_node(rs, o10, 0u);
  f.c[2] = load_node(rs, o01, 0u);
  f.c[3] = load_node(rs, o11, 0u);
  f.c[4] = load_node(rs, o00 + 64u, 0u);
  f.c[5] = load_node(rs, o10 + 64u, 0u);
  f.c[6] = load_node(rs, o01 + 64u, 0u);
  f.c[7] = load_node(rs, o11 + 64u, 0u);
  const float4* c = f.c;
  f.phi = tri(c[0].x, c[1].x, c[2].x, c[3].x, c[4].x, c[5].x, c[6].x, c[7].x, f.tx, f.ty, f.tz);
  if (!(f.phi < 0.f)) return;
  f.contact = true;
  f.gx = tri(c[0].y, c[1].y, c[2].y, c[3].y, c[4].y, c[5].y, c[6].y, c[7].y, f.tx, f.ty, f.tz);
  f.gy = tri(c[0].z, c[1].z, c[2].z, c[3].z, c[4].z, c[5].z, c[6].z, c[7].z, f.tx, f.ty, f.tz);
  f.gz = tri(c[0].w, c[1].w, c[2].w, c[3].w, c[4].w, c[5].w, c[6].w, c[7].w, f.tx, f.ty, f.tz);
  const float gg = fmaf(f.gx, f.gx, fmaf(f.gy, f.gy, f.gz * f.gz));
  if (!(gg >= 1e-12f)) return;
  f.force = true;
  f.r = __builtin_amdgcn_rsqf(gg);  // hardware reciprocal square root (~1 ulp)
  f.nox = f.gx * f.r;
  f.noy = f.gy * f.r;
  f.noz = f.gz * f.r;
  // pad-frame normal n = R^T n_o = h A^T n_o
  const float hx = x.h;
  f.n[0] = hx * fmaf(x.A[0], f.nox, fmaf(x.A[3], f.noy, x.A[6] * f.noz));
  f.n[1] = hx * fmaf(x.A[1], f.nox, fmaf(x.A[4], f.noy, x.A[7] * f.noz));
  f.n[2] = hx * fmaf(x.A[2], f.nox, fmaf(x.A[5], f.noy, x.A[8] * f.noz));
  // relative velocity x_dot = V + W x p
  f.v[0] = x.V[0] + fmaf(x.W[1], pz, -x.W[2] * py);
  f.v[1] = x.V[1] + fmaf(x.W[2], px, -x.W[0] * pz);
  f.v[2] = x.V[2] + fmaf(x.W[0], py, -x.W[1] * px);
  f.dd = fmaf(f.n[0], f.v[0], fmaf(f.n[1], f.v[1], f.n[2] * f.v[2]));
  // normal law s = (-k_n + k_d d_dot) w: w = phi (Section III-C), or with
  // an exponent p != 1, w = -(-phi)^p (the nonlinear variant of Section VII)
  f.w = f.phi;
  f.dw = 1.f;
  if constexpr (NL) {
    const float dl = -f.phi;
    const float dp = exp2f(x.hc * log2f(dl));
    f.w = -dp;
    f.dw = x.hc * dp / dl;
  }
  f.s = fmaf(x.prm[1], f.dd, -x.prm[0]) * f.w;
  for (int a = 0; a < 3; ++a) {
    f.fn[a] = f.s * f.n[a];
    f.vt[a] = fmaf(-f.dd, f.n[a], f.v[a]);
  }
  // hardware square root and reciprocal (~1 ulp each); slipping implies |v_t| > 0
  f.vtn = __builtin_amdgcn_sqrtf(fmaf(f.vt[0], f.vt[0], fmaf(f.vt[1], f.vt[1], f.vt[2] * f.vt[2])));
  f.cap = x.prm[3] * fabsf(f.s);
  f.stick = x.prm[2] * f.vtn <= f.cap;
  const float coef = f.stick ? -x.prm[2] : -f.cap * __builtin_amdgcn_rcpf(f.vtn);
  for (int a = 0; a < 3; ++a) f.ft[a] = coef * f.vt[a];
}

// Next execution slot of a tile loop (uniform across the workgroup).
template <int BLOCK>
__device__ __forceinline__ int next_slot(int slot, int dynamic, int32_t* queue, int* s_next) {
  if (dynamic) {
    if (threadIdx.x == 0) *s_next = (int)gridDim.x + atomicAdd(queue, 1);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*s_next);
  }
  __syncthreads();
  return slot + (int)gridDim.x;
}

// ---------------------------------------------------------------------------
// Forward kernel.
// ---------------------------------------------------------------------------
// Tile records are read at a workgroup-uniform index through restrict
// (read-only, non-aliased) pointers, so they land in scalar registers and the
// buffer resource of the grid is uniform (no per-lane waterfall).
// Output pointers of one tile (SoA, taxel k of the tile at element k).
struct TileOut {
  float *d, *n0, *n1, *n2, *f0, *f1, *f2, *t0, *t1, *t2;
};

// One taxel of the forward path: evaluation, optional SoA stores, wrench
// accumulation.  Returns the observation channels (|f_n|, f_t,x, f_t,y).
template <bool FIELDS, bool NL>
__device__ __forceinline__ void taxel_step(const InstXf& x, const InstStatic& st, __amdgpu_buffer_rsrc_t rs,
                                           const float* tx, const float* ty, const float* tz, uint32_t k,
                                           const TileOut& o, float acc[6], float ch[3]) {
  // uniform 64-bit base + 32-bit lane offset: saddr addressing, no 64-bit VALU math
  const float px = at(tx, k), py = at(ty, k), pz = at(tz, k);
  TaxelFwd f;
  taxel_forward<NL>(x, st, rs, px, py, pz, f);
  float dep = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
  float fn0 = 0.f, fn1 = 0.f, fn2 = 0.f, ft0 = 0.f, ft1 = 0.f, ft2 = 0.f, sn = 0.f;
  if (f.contact) dep = -f.phi;
  if (f.force) {
    n0 = f.n[0]; n1 = f.n[1]; n2 = f.n[2];
    fn0 = f.fn[0]; fn1 = f.fn[1]; fn2 = f.fn[2];
    ft0 = f.ft[0]; ft1 = f.ft[1]; ft2 = f.ft[2];
    sn = fabsf(f.s);
  }
  if constexpr (FIELDS) {
    put(o.d, k, dep);
    put(o.n0, k, n0); put(o.n1, k, n1); put(o.n2, k, n2);
    put(o.f0, k, fn0); put(o.f1, k, fn1); put(o.f2, k, fn2);
    put(o.t0, k, ft0); put(o.t1, k, ft1); put(o.t2, k, ft2);
  }
  const float F0 = fn0 + ft0, F1 = fn1 + ft1, F2 = fn2 + ft2;
  acc[0] += F0;
  acc[1] += F1;
  acc[2] += F2;
  acc[3] += fmaf(py, F2, -pz * F1);
  acc[4] += fmaf(pz, F0, -px * F2);
  acc[5] += fmaf(px, F1, -py * F0);
  ch[0] = sn;
  ch[1] = ft0;
  ch[2] = ft1;
}

// Deterministic per-wave pooling: for each distinct bin among the lanes (in
// order of the lowest lane holding it) the lanes of that bin are summed with
// a fixed butterfly and lane 0 adds the sums to the wave's accumulator row.
// Needs every lane of the wave active; b < 0 means no bin.
__device__ __forceinline__ void pool_wave(float* acc, int lane, int b, const float ch[3]) {
  uint64_t pending = __ballot(b >= 0);
  while (pending) {
    const int lead = __ffsll((unsigned long long)pending) - 1;
    const int bb = __builtin_amdgcn_readlane(b, lead);
    const bool mine = b == bb;
    const float s0 = wave_sum(mine ? ch[0] : 0.f);
    const float s1 = wave_sum(mine ? ch[1] : 0.f);
    const float s2 = wave_sum(mine ? ch[2] : 0.f);
    if (lane == 0) {
      acc[3 * bb] += s0;
      acc[3 * bb + 1] += s1;
      acc[3 * bb + 2] += s2;
    }
    pending &= ~__ballot(mine);
  }
}

// MODE bits: kFields writes the per-taxel SoA fields; kObserve pools the
// observation channels per bin into per-tile partials (dynamic LDS of
// BLOCK/64 * obs_n * 3 floats); kNonlinear selects the nonlinear normal law;
// kFused computes each tile's pad record in the kernel (wave 0, shared through
// LDS) instead of reading the prologue's, so a call is one launch.
constexpr int kFields = 1;
constexpr int kObserve = 2;
constexpr int kNonlinear = 4;
constexpr int kFused = 8;

// A record made uniform: every dword through the scalar unit.
__device__ __forceinline__ InstXf uniform_record(const InstXf& v) {
  InstXf u;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&v);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&u);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(InstXf) / 4); ++k) dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
  return u;
}

template <int BLOCK, int MODE>
__global__ __launch_bounds__(BLOCK) void k_force_fwd(
    const Tile* __restrict__ tiles, const int32_t* __restrict__ order, int32_t n_tiles, int32_t dynamic,
    int32_t* __restrict__ queue, const InstStatic* __restrict__ stat, const InstXf* __restrict__ xfs,
    const float* __restrict__ tmpl, int64_t tmpl_T, float* __restrict__ depth, float* __restrict__ normal,
    float* __restrict__ fn, float* __restrict__ ft, int64_t T, float* __restrict__ partial,
    const int32_t* __restrict__ obs_bin, int32_t obs_n, float* __restrict__ obs_partial, const FusedIn fin) {
  constexpr int NW = BLOCK / 64;
  constexpr bool FIELDS = (MODE & kFields) != 0;
  constexpr bool NL = (MODE & kNonlinear) != 0;
  constexpr bool FUSED = (MODE & kFused) != 0;
  __shared__ float red[NW][6];
  __shared__ int s_next;
  __shared__ InstXf s_rec;  // kFused: the tile's pad record
  extern __shared__ float obs_acc[];  // [NW][obs_n * 3], kObserve only
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int slot = blockIdx.x;
  while (slot < n_tiles) {
    const int tid = __builtin_amdgcn_readfirstlane(order[slot]);
    const Tile tl = tiles[tid];
    const InstStatic st = stat[tl.inst];
    InstXf x;
    if constexpr (FUSED) {
      if (wave == 0) {
        InstXf r;
        uint32_t bits = 0;
        // the environment comes with the tile, so the pose loads need not wait for the pad's static record
        pad_record(fin.pad_pose, fin.obj_pose, fin.pad_twist, fin.obj_twist, fin.params, fin.obj_pose_delta, st,
                   tl.inst, tl.env, fin.hc, r, bits);
        if (lane == 0) {
          s_rec = r;
          if (bits && fin.status && tl.k0 == 0) atomicOr(fin.status, bits);  // once per pad
        }
      }
      __syncthreads();
      x = uniform_record(s_rec);
    } else {
      x = xfs[tl.inst];
    }
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(st.grid, st.grid_bytes);
    const float* tx = tmpl + st.tmpl_off + tl.k0;
    const float* ty = tx + tmpl_T;
    const float* tz = ty + tmpl_T;
    TileOut o{};
    if constexpr (FIELDS) {
      const int64_t ob = st.out_off + tl.k0;
      o.d = depth + ob;
      o.n0 = normal + ob;
      o.n1 = o.n0 + T;
      o.n2 = o.n1 + T;
      o.f0 = fn + ob;
      o.f1 = o.f0 + T;
      o.f2 = o.f1 + T;
      o.t0 = ft + ob;
      o.t1 = o.t0 + T;
      o.t2 = o.t1 + T;
    }
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float ch[3];
    if constexpr ((MODE & kObserve) != 0) {
      const int row = obs_n * 3;
      for (int j = threadIdx.x; j < NW * row; j += BLOCK) obs_acc[j] = 0.f;
      __syncthreads();
      const int32_t* bins = obs_bin + st.tmpl_off + tl.k0;
      // whole-block strides so that every lane takes part in the pooling
      for (uint32_t base = 0; base < (uint32_t)tl.count; base += BLOCK) {
        const uint32_t k = base + threadIdx.x;
        int b = -1;
        ch[0] = ch[1] = ch[2] = 0.f;
        if (k < (uint32_t)tl.count) {
          taxel_step<FIELDS, NL>(x, st, rs, tx, ty, tz, k, o, acc, ch);
          b = bins[k];
        }
        pool_wave(obs_acc + wave * row, lane, b, ch);
      }
    } else {
      for (uint32_t k = threadIdx.x; k < (uint32_t)tl.count; k += BLOCK)
        taxel_step<FIELDS, NL>(x, st, rs, tx, ty, tz, k, o, acc, ch);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float v = wave_sum(acc[c]);
      if (lane == 0) red[wave][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
      float s = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += red[w][threadIdx.x];
      partial[6 * (int64_t)tid + threadIdx.x] = s;
    }
    if constexpr ((MODE & kObserve) != 0) {
      const int row = obs_n * 3;
      float* dst = obs_partial + (int64_t)tid * row;
      for (int j = threadIdx.x; j < row; j += BLOCK) {
        float s = 0.f;
        for (int w = 0; w < NW; ++w) s += obs_acc[w * row + j];
        dst[j] = s;
      }
    }
    slot = next_slot<BLOCK>(slot, dynamic, queue, &s_next);
  }
}

// Observation of each pad: the pad's tile partials summed in tile order,
// divided by the bin's taxel count and the channel scale, clipped.
__global__ __launch_bounds__(256) void k_obs_reduce(const ObsReduceArgs a) {
  const int row = a.obs_n * 3;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)a.n_inst * row) return;
  const int i = (int)(idx / row);
  const int j = (int)(idx - (int64_t)i * row);
  float s = 0.f;
  for (int64_t t = a.inst_tile_begin[i]; t < a.inst_tile_begin[i + 1]; ++t) s += a.partial[t * row + j];
  const int c = j % 3;
  float v = s * a.icnt[(int64_t)a.inst_tmpl[i] * a.obs_n + j / 3] / a.scale[c];
  if (a.clip > 0.f) v = fminf(fmaxf(v, -a.clip), a.clip);
  a.obs[idx] = v;
}

__global__ __launch_bounds__(256) void k_wrench_reduce(WrenchReduceArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n_inst) return;
  float s[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int64_t t = a.inst_tile_begin[i]; t < a.inst_tile_begin[i + 1]; ++t)
    for (int c = 0; c < 6; ++c) s[c] += a.partial[6 * t + c];
  for (int c = 0; c < 6; ++c) a.wrench[6 * (int64_t)i + c] = s[c];
}

// ---------------------------------------------------------------------------
// Adjoint kernel: recompute the forward per taxel, then reverse mode of
// L = w_fn . f_n + w_ft . f_t.  Per-lane accumulators (pad/object frames):
//   P1 = sum x_dot_bar, P2 = sum x_dot_bar x x_p, N1 = sum n x n_bar,
//   U1 = sum u_bar,     U2 = sum u_bar x u       (grid coordinates),
//   and the four parameter adjoints.  k_grad_reduce maps them to the world.
// ---------------------------------------------------------------------------
template <int BLOCK, bool NL>
__global__ __launch_bounds__(BLOCK) void k_force_bwd(
    const Tile* __restrict__ tiles, const int32_t* __restrict__ order, int32_t n_tiles, int32_t dynamic,
    int32_t* __restrict__ queue, const InstStatic* __restrict__ stat, const InstXf* __restrict__ xfs,
    const float* __restrict__ tmpl, int64_t tmpl_T, const float* __restrict__ w_fn,
    const float* __restrict__ w_ft, int64_t T, double* __restrict__ partial) {
  constexpr int NW = BLOCK / 64;
  __shared__ double red[NW][kBwdAcc];
  __shared__ int s_next;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int slot = blockIdx.x;
  while (slot < n_tiles) {
    const int tid = __builtin_amdgcn_readfirstlane(order[slot]);
    const Tile tl = tiles[tid];
    const InstStatic st = stat[tl.inst];
    const InstXf x = xfs[tl.inst];
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(st.grid, st.grid_bytes);
    const float* tx = tmpl + st.tmpl_off + tl.k0;
    const float* ty = tx + tmpl_T;
    const float* tz = ty + tmpl_T;
    const int64_t ob = st.out_off + tl.k0;
    const float* wa0 = w_fn + ob;
    const float* wa1 = wa0 + T;
    const float* wa2 = wa1 + T;
    const float* wb0 = w_ft + ob;
    const float* wb1 = wb0 + T;
    const float* wb2 = wb1 + T;
    const float kn = x.prm[0], kd = x.prm[1], kt = x.prm[2], mu = x.prm[3];
    float acc[kBwdAcc];
#pragma unroll
    for (int c = 0; c < kBwdAcc; ++c) acc[c] = 0.f;
    for (uint32_t k = threadIdx.x; k < (uint32_t)tl.count; k += BLOCK) {
      const float px = at(tx, k), py = at(ty, k), pz = at(tz, k);
      // the loss weights are requested with the template point, so that their
      // latency overlaps the forward recomputation instead of following it
      const float A[3] = {at(wa0, k), at(wa1, k), at(wa2, k)};
      const float B[3] = {at(wb0, k), at(wb1, k), at(wb2, k)};
      TaxelFwd f;
      taxel_forward<NL>(x, st, rs, px, py, pz, f);
      if (!f.force) continue;
      // f_n = s n
      float nb[3], vb[3], vtb[3];
      for (int c = 0; c < 3; ++c) nb[c] = f.s * A[c];
      float sb = A[0] * f.n[0] + A[1] * f.n[1] + A[2] * f.n[2];
      float ktb = 0.f, mub = 0.f;
      if (f.stick) {  // f_t = -k_t v_t
        for (int c = 0; c < 3; ++c) vtb[c] = -kt * B[c];
        ktb = -(B[0] * f.vt[0] + B[1] * f.vt[1] + B[2] * f.vt[2]);
      } else {  // f_t = -cap v_t / |v_t|
        const float iv = 1.f / f.vtn;
        const float q = f.cap * iv;
        const float vh[3] = {f.vt[0] * iv, f.vt[1] * iv, f.vt[2] * iv};
        const float bv = B[0] * vh[0] + B[1] * vh[1] + B[2] * vh[2];
        for (int c = 0; c < 3; ++c) vtb[c] = -q * (B[c] - bv * vh[c]);
        const float capb = -bv;
        mub = capb * fabsf(f.s);
        sb += capb * mu * (f.s < 0.f ? -1.f : 1.f);
      }
      // v_t = x_dot - d_dot n
      float ddb = -(vtb[0] * f.n[0] + vtb[1] * f.n[1] + vtb[2] * f.n[2]);
      for (int c = 0; c < 3; ++c) {
        vb[c] = vtb[c];
        nb[c] -= f.dd * vtb[c];
      }
      // s = (-k_n + k_d d_dot) w(phi)
      const float knb = -f.w * sb;
      const float kdb = f.dd * f.w * sb;
      ddb += kd * f.w * sb;
      const float phib = (kd * f.dd - kn) * sb * f.dw;
      // d_dot = n . x_dot
      for (int c = 0; c < 3; ++c) {
        nb[c] += ddb * f.v[c];
        vb[c] += ddb * f.n[c];
      }
      // x_dot = V + W x p
      acc[0] += vb[0]; acc[1] += vb[1]; acc[2] += vb[2];
      acc[3] += vb[1] * pz - vb[2] * py;
      acc[4] += vb[2] * px - vb[0] * pz;
      acc[5] += vb[0] * py - vb[1] * px;
      // rotation of the normal: N1 += n x n_bar
      acc[6] += f.n[1] * nb[2] - f.n[2] * nb[1];
      acc[7] += f.n[2] * nb[0] - f.n[0] * nb[2];
      acc[8] += f.n[0] * nb[1] - f.n[1] * nb[0];
      // n = R^T n_o  ->  n_o_bar = R n_bar = h A n_bar
      const float nob0 = x.h * (x.A[0] * nb[0] + x.A[1] * nb[1] + x.A[2] * nb[2]);
      const float nob1 = x.h * (x.A[3] * nb[0] + x.A[4] * nb[1] + x.A[5] * nb[2]);
      const float nob2 = x.h * (x.A[6] * nb[0] + x.A[7] * nb[1] + x.A[8] * nb[2]);
      // n_o = g / |g|
      const float pr = nob0 * f.nox + nob1 * f.noy + nob2 * f.noz;
      const float gb0 = f.r * (nob0 - pr * f.nox);
      const float gb1 = f.r * (nob1 - pr * f.noy);
      const float gb2 = f.r * (nob2 - pr * f.noz);
      // phi, g trilinear in t: corner scalars Q = phi_bar Phi_c + g_bar . G_c
      float Q[8];
#pragma unroll
      for (int c = 0; c < 8; ++c)
        Q[c] = phib * f.c[c].x + gb0 * f.c[c].y + gb1 * f.c[c].z + gb2 * f.c[c].w;
      const float ub0 = lerp(lerp(Q[1] - Q[0], Q[3] - Q[2], f.ty), lerp(Q[5] - Q[4], Q[7] - Q[6], f.ty), f.tz);
      const float ub1 = lerp(lerp(Q[2] - Q[0], Q[3] - Q[1], f.tx), lerp(Q[6] - Q[4], Q[7] - Q[5], f.tx), f.tz);
      const float ub2 = lerp(lerp(Q[4] - Q[0], Q[5] - Q[1], f.tx), lerp(Q[6] - Q[2], Q[7] - Q[3], f.tx), f.ty);
      acc[9] += ub0; acc[10] += ub1; acc[11] += ub2;
      acc[12] += ub1 * f.uz - ub2 * f.uy;
      acc[13] += ub2 * f.ux - ub0 * f.uz;
      acc[14] += ub0 * f.uy - ub1 * f.ux;
      acc[15] += knb; acc[16] += kdb; acc[17] += ktb; acc[18] += mub;
    }
#pragma unroll
    for (int c = 0; c < kBwdAcc; ++c) {
      const double v = wave_sum((double)acc[c]);
      if (lane == 0) red[wave][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < kBwdAcc) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += red[w][threadIdx.x];
      partial[kBwdAcc * (int64_t)tid + threadIdx.x] = s;
    }
    slot = next_slot<BLOCK>(slot, dynamic, queue, &s_next);
  }
}

__device__ void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ void matvec(const double R[9], const double v[3], double o[3]) {
  for (int r = 0; r < 3; ++r) o[r] = R[3 * r] * v[0] + R[3 * r + 1] * v[1] + R[3 * r + 2] * v[2];
}

// Per environment (FP64): world-frame gradients
//   dt     = -R_o U1/h + (R_p P1) x w_o
//   dtheta =  R_p N1 + R_o X2,  X2 = (U1 x origin)/h + U2
//   dv_o   = -R_p P1
//   dw_o   =  R_p (P2 + P1 x c_p),  c_p = R_p^T (t_p - t_o)
// summed over the environment's pads; then the rotation block is mapped from
// a left perturbation of the composed pose to the input delta: J_l(delta)^T.
__global__ __launch_bounds__(64) void k_grad_reduce(GradReduceArgs a) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n_env) return;
  double gp[6] = {0, 0, 0, 0, 0, 0}, gt[6] = {0, 0, 0, 0, 0, 0}, gk[4] = {0, 0, 0, 0};
  uint32_t bits = 0;
  double Ro[9], to[3];
  const float* dl = a.obj_pose_delta ? a.obj_pose_delta + 6 * (int64_t)e : nullptr;
  const bool ok_o = object_pose(a.obj_pose + 7 * (int64_t)e, dl, Ro, to, bits);
  const double wo[3] = {a.obj_twist[6 * (int64_t)e + 3], a.obj_twist[6 * (int64_t)e + 4],
                        a.obj_twist[6 * (int64_t)e + 5]};
  for (int32_t q = a.env_inst_begin[e]; q < a.env_inst_begin[e + 1] && ok_o; ++q) {
    const int i = a.env_inst[q];
    double S[kBwdAcc];
    for (int c = 0; c < kBwdAcc; ++c) S[c] = 0.0;
    for (int64_t t = a.inst_tile_begin[i]; t < a.inst_tile_begin[i + 1]; ++t)
      for (int c = 0; c < kBwdAcc; ++c) S[c] += a.partial[kBwdAcc * t + c];
    double Rp[9];
    const float* pp = a.pad_pose + 7 * (int64_t)i;
    if (!quat_to_R(pp, Rp, bits)) continue;
    const InstStatic st = a.stat[i];
    const double h = st.h;
    const double org[3] = {st.ox, st.oy, st.oz};
    const double P1[3] = {S[0], S[1], S[2]}, P2[3] = {S[3], S[4], S[5]}, N1[3] = {S[6], S[7], S[8]};
    const double U1[3] = {S[9], S[10], S[11]}, U2[3] = {S[12], S[13], S[14]};
    double X1[3], X2[3], tmp[3], tmp2[3];
    for (int c = 0; c < 3; ++c) X1[c] = U1[c] / h;
    cross3(U1, org, tmp);
    for (int c = 0; c < 3; ++c) X2[c] = tmp[c] / h + U2[c];
    double RpP1[3], RoX1[3], RoX2[3], RpN1[3];
    matvec(Rp, P1, RpP1);
    matvec(Ro, X1, RoX1);
    matvec(Ro, X2, RoX2);
    matvec(Rp, N1, RpN1);
    cross3(RpP1, wo, tmp);
    for (int c = 0; c < 3; ++c) {
      gp[c] += -RoX1[c] + tmp[c];
      gp[3 + c] += RpN1[c] + RoX2[c];
      gt[c] += -RpP1[c];
    }
    const double d[3] = {pp[4] - to[0], pp[5] - to[1], pp[6] - to[2]};
    const double cp[3] = {Rp[0] * d[0] + Rp[3] * d[1] + Rp[6] * d[2], Rp[1] * d[0] + Rp[4] * d[1] + Rp[7] * d[2],
                          Rp[2] * d[0] + Rp[5] * d[1] + Rp[8] * d[2]};
    cross3(P1, cp, tmp);
    for (int c = 0; c < 3; ++c) tmp[c] += P2[c];
    matvec(Rp, tmp, tmp2);
    for (int c = 0; c < 3; ++c) gt[3 + c] += tmp2[c];
    for (int c = 0; c < 4; ++c) gk[c] += S[15 + c];
  }
  if (dl) {  // dL/d(delta_theta) = J_l(delta_theta)^T dL/d(left perturbation)
    const double p[3] = {dl[3], dl[4], dl[5]};
    const double t2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    double a1, a2;
    if (t2 < 1e-12) {
      a1 = 0.5 - t2 / 24.0;
      a2 = 1.0 / 6.0 - t2 / 120.0;
    } else {
      const double t = sqrt(t2);
      a1 = (1.0 - cos(t)) / t2;
      a2 = (t - sin(t)) / (t2 * t);
    }
    // J_l = I + a1 K + a2 K^2, K = [p]x ; J_l^T g = g - a1 K g + a2 K^2 g
    const double g[3] = {gp[3], gp[4], gp[5]};
    double Kg[3], KKg[3];
    cross3(p, g, Kg);
    cross3(p, Kg, KKg);
    for (int c = 0; c < 3; ++c) gp[3 + c] = g[c] - a1 * Kg[c] + a2 * KKg[c];
  }
  for (int c = 0; c < 6; ++c) {
    a.g_obj_pose[6 * (int64_t)e + c] = (float)gp[c];
    a.g_obj_twist[6 * (int64_t)e + c] = (float)gt[c];
  }
  for (int c = 0; c < 4; ++c) a.g_params[4 * (int64_t)e + c] = (float)gk[c];
}

// Fill n 32-bit words with zero (a kernel, not a memset, so that it also
// replays correctly inside captured graphs).
__global__ __launch_bounds__(256) void k_zero_u32(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Device scratch of the allocation-free forward entry point: one static
// array per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address resolved below, once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Object poses after moving for time t at a constant twist (FP64): origin at
// t_o + v t, orientation Exp(w t) R_o (w the world-frame angular velocity),
// i.e. q(t) = q_w(t) q_0 with q_w = (cos(|w| t / 2), sin(|w| t / 2) w / |w|).
__global__ __launch_bounds__(256) void k_pose_step(const float* __restrict__ pose0, const float* __restrict__ twist,
                                                   double t, int32_t n_env, float* __restrict__ pose) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n_env) return;
  const float* p = pose0 + 7 * (int64_t)e;
  const float* w = twist + 6 * (int64_t)e;
  float* o = pose + 7 * (int64_t)e;
  for (int a = 0; a < 3; ++a) o[4 + a] = (float)((double)p[4 + a] + (double)w[a] * t);
  const double rx = (double)w[3] * t, ry = (double)w[4] * t, rz = (double)w[5] * t;
  const double ang = sqrt(rx * rx + ry * ry + rz * rz);
  const double half = 0.5 * ang;
  // sin(|a| / 2) / |a|, by its series below 1e-4 (error < 1e-18)
  const double s = ang < 1e-4 ? 0.5 - ang * ang / 48.0 : sin(half) / ang;
  const double w1 = cos(half), x1 = s * rx, y1 = s * ry, z1 = s * rz;
  const double w2 = p[0], x2 = p[1], y2 = p[2], z2 = p[3];
  o[0] = (float)(w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2);
  o[1] = (float)(w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2);
  o[2] = (float)(w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2);
  o[3] = (float)(w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2);
}

}  // namespace

hipError_t launch_pose_step(const float* pose0, const float* twist, double t, int32_t n_env, float* pose,
                            hipStream_t stream) {
  if (n_env <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pose_step, dim3((unsigned)((n_env + 255) / 256)), dim3(256), 0, stream, pose0, twist, t, n_env,
                     pose);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t scratch_address(int device, void** out) {
  static std::mutex mu;
  static void* addr[kMaxScratchDevices] = {};
  *out = nullptr;
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t launch_prepare_grid(const float* phi, float4* out, int nx, int ny, int nz, float h, uint32_t* bad,
                               hipStream_t stream) {
  const int64_t n = (int64_t)nx * ny * nz;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_prepare_grid, dim3((unsigned)blocks), dim3(256), 0, stream, phi, out, nx, ny, nz, h, bad);
  return hipGetLastError();
}

hipError_t launch_clear_mask(const float* phi, uint32_t* mask, int nx, int ny, int nz, hipStream_t stream) {
  const MaskDims m = mask_dims(nx, ny, nz);
  const int64_t n = m.wx * m.wy * m.wz;
  hipLaunchKernelGGL(k_clear_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, phi, mask, nx, ny, nz,
                     (int)m.wx, (int)m.wy, (int)m.wz);
  return hipGetLastError();
}

hipError_t launch_prologue(const PrologueArgs& a, hipStream_t stream) {
  const int blocks = a.n_inst > 0 ? (a.n_inst + 63) / 64 : 1;
  hipLaunchKernelGGL(k_prologue, dim3(blocks), dim3(64), 0, stream, a);
  return hipGetLastError();
}

#define TACSL_FWD_ARGS                                                                                  \
  a.tiles, a.order, a.n_tiles, a.dynamic, a.queue, a.stat, a.xf, a.tmpl, a.tmpl_T, a.depth, a.normal, a.fn, \
      a.ft, a.T, a.partial, a.obs_bin, a.obs_n, a.obs_partial, a.fin

template <int MODE>
hipError_t launch_forward_mode(const FwdArgs& a, int block, int grid, hipStream_t stream) {
  const size_t lds = (MODE & kObserve) ? (size_t)(block / 64) * a.obs_n * 3 * sizeof(float) : 0;
  switch (block) {
    case 64: hipLaunchKernelGGL((k_force_fwd<64, MODE>), dim3(grid), dim3(64), lds, stream, TACSL_FWD_ARGS); break;
    case 128: hipLaunchKernelGGL((k_force_fwd<128, MODE>), dim3(grid), dim3(128), lds, stream, TACSL_FWD_ARGS); break;
    case 256: hipLaunchKernelGGL((k_force_fwd<256, MODE>), dim3(grid), dim3(256), lds, stream, TACSL_FWD_ARGS); break;
    case 512: hipLaunchKernelGGL((k_force_fwd<512, MODE>), dim3(grid), dim3(512), lds, stream, TACSL_FWD_ARGS); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_forward(const FwdArgs& a, int block, int grid, hipStream_t stream) {
  if (a.fused && (a.mode != kFields || a.dynamic)) return hipErrorInvalidValue;
  switch (a.mode | (a.nonlinear ? kNonlinear : 0) | (a.fused ? kFused : 0)) {
    case kFields: return launch_forward_mode<kFields>(a, block, grid, stream);
    case kFields | kFused: return launch_forward_mode<kFields | kFused>(a, block, grid, stream);
    case kFields | kNonlinear | kFused: return launch_forward_mode<kFields | kNonlinear | kFused>(a, block, grid, stream);
    case kObserve: return launch_forward_mode<kObserve>(a, block, grid, stream);
    case kFields | kObserve: return launch_forward_mode<kFields | kObserve>(a, block, grid, stream);
    case kFields | kNonlinear: return launch_forward_mode<kFields | kNonlinear>(a, block, grid, stream);
    case kObserve | kNonlinear: return launch_forward_mode<kObserve | kNonlinear>(a, block, grid, stream);
    case kFields | kObserve | kNonlinear:
      return launch_forward_mode<kFields | kObserve | kNonlinear>(a, block, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_spatial_order(const SpatialArgs& a, hipStream_t stream) {
  if (a.n_inst == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sp_scan, dim3(1), dim3(1024), 0, stream, a);
  hipLaunchKernelGGL(k_sp_place, dim3((unsigned)((a.n_inst + 255) / 256)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_obs_reduce(const ObsReduceArgs& a, hipStream_t stream) {
  const int64_t n = (int64_t)a.n_inst * a.obs_n * 3;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_obs_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_wrench_reduce(const WrenchReduceArgs& a, hipStream_t stream) {
  const int blocks = (a.n_inst + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_wrench_reduce, dim3(blocks), dim3(256), 0, stream, a);
  return hipGetLastError();
}

#define TACSL_BWD_ARGS \
  a.tiles, a.order, a.n_tiles, a.dynamic, a.queue, a.stat, a.xf, a.tmpl, a.tmpl_T, a.w_fn, a.w_ft, a.T, a.partial

template <bool NL>
hipError_t launch_backward_law(const BwdArgs& a, int block, int grid, hipStream_t stream) {
  switch (block) {
    case 64: hipLaunchKernelGGL((k_force_bwd<64, NL>), dim3(grid), dim3(64), 0, stream, TACSL_BWD_ARGS); break;
    case 128: hipLaunchKernelGGL((k_force_bwd<128, NL>), dim3(grid), dim3(128), 0, stream, TACSL_BWD_ARGS); break;
    case 256: hipLaunchKernelGGL((k_force_bwd<256, NL>), dim3(grid), dim3(256), 0, stream, TACSL_BWD_ARGS); break;
    case 512: hipLaunchKernelGGL((k_force_bwd<512, NL>), dim3(grid), dim3(512), 0, stream, TACSL_BWD_ARGS); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_backward(const BwdArgs& a, int block, int grid, hipStream_t stream) {
  return a.nonlinear ? launch_backward_law<true>(a, block, grid, stream)
                     : launch_backward_law<false>(a, block, grid, stream);
}

hipError_t launch_grad_reduce(const GradReduceArgs& a, hipStream_t stream) {
  const int blocks = (a.n_env + 63) / 64;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_reduce, dim3(blocks), dim3(64), 0, stream, a);
  return hipGetLastError();
}

}  // namespace tacsl
