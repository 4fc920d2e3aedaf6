// Tactile depth image kernels of libtacsl for gfx950 (MI355X), and the
// local slope bounds the ray march relies on.
#include <hip/hip_runtime.h>

#include "tacsl.h"
#include "tacsl_device.h"
#include "tacsl_internal.h"

namespace tacsl {
namespace {

// ---------------------------------------------------------------------------
// Tactile depth image (Section III-B).  A camera behind the gel looks along
// +z of the pad frame; pixel (r, c) looks through the pad-plane point
// P = (x0 + (c + 1/2) dx, y0 + (r + 1/2) dy, 0), from a pinhole at
// (0, 0, -cam_dist) or along +z (orthographic).  Parametrized by its height
// z, the ray is X(z) = P + z (P_x / D, P_y / D, 1) (pinhole) or P + z e_z, so
// its grid coordinates are affine in z: u(z) = u0 + z uz.  The pixel reads
// cam_dist + the height of the first point of [-gel, 0] (clipped to the node
// box) where the trilinear phi <= 0, or cam_dist (the gel surface).
//
// The ray advances cell by cell.  Far from the surface it takes sphere-tracing
// steps: near the current block, |d phi / dz| <= sum_k m_k |duk/dz| with m_k
// the block's slope bounds (per grid step, see DepthGrid), so a step of phi
// over that sum, kept within 7 cells so that it stays near the block, cannot
// pass the surface; it is taken whenever it reaches past the current cell.  Otherwise the rest of the cell is searched exactly:
// along the ray the trilinear field is a cubic in z, monotone between the
// roots of its derivative, so its sign (direct trilinear form) at those points
// and at the cell exit brackets the first root, which safeguarded Newton steps
// on the cubic then refine.
// Every iteration moves past at least one grid plane, so the work per ray is
// bounded by the planes it crosses.
// ---------------------------------------------------------------------------
constexpr int kDepthMaxIter = 4096;

__device__ __forceinline__ float load_phi(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

struct RayCell {
  int cx, cy, cz;
  float a[8];  // corner phi, index dx + 2 dy + 4 dz
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc_f(const float* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0, (int)bytes, kBufferFlags);
}

__device__ __forceinline__ void ray_cell(const InstStatic& st, const DepthGrid& g, __amdgpu_buffer_rsrc_t rs,
                                         RayCell& rc, float ux, float uy, float uz) {
  // clamped on both sides: points on the box faces, and rounding just outside
  const int cx = min(max((int)floorf(ux), 0), st.nx - 2);
  const int cy = min(max((int)floorf(uy), 0), st.ny - 2);
  const int cz = min(max((int)floorf(uz), 0), st.nz - 2);
  if (cx == rc.cx && cy == rc.cy && cz == rc.cz) return;
  rc.cx = cx;
  rc.cy = cy;
  rc.cz = cz;
  // x-quad columns: the two x-nodes by per-lane offsets, y by a scalar
  // offset, z by an immediate offset
  const uint32_t yz = __umul24((uint32_t)cy, g.stride_y) + (uint32_t)cz * 16u;
  const uint32_t x0 = (uint32_t)cx, x1 = x0 + 1u;
  const uint32_t o0 = __umul24(x0 >> 2, g.stride_q) + (x0 & 3u) * 4u + yz;
  const uint32_t o1 = __umul24(x1 >> 2, g.stride_q) + (x1 & 3u) * 4u + yz;
  const uint32_t sy = g.stride_y;
  rc.a[0] = load_phi(rs, o0, 0u);
  rc.a[1] = load_phi(rs, o1, 0u);
  rc.a[2] = load_phi(rs, o0, sy);
  rc.a[3] = load_phi(rs, o1, sy);
  rc.a[4] = load_phi(rs, o0 + 16u, 0u);
  rc.a[5] = load_phi(rs, o1 + 16u, 0u);
  rc.a[6] = load_phi(rs, o0 + 16u, sy);
  rc.a[7] = load_phi(rs, o1 + 16u, sy);
}

__device__ __forceinline__ float cell_tri(const RayCell& rc, float tx, float ty, float tz) {
  return tri(rc.a[0], rc.a[1], rc.a[2], rc.a[3], rc.a[4], rc.a[5], rc.a[6], rc.a[7], tx, ty, tz);
}

// Height of the next grid plane of one axis strictly above z (iuz = 1 / uz).
// A crossing height that rounds onto z moves on to the following plane.
__device__ __forceinline__ float next_plane(float u0, float uz, float iuz, float z) {
  if (uz == 0.f) return INFINITY;
  const float dir = uz > 0.f ? 1.f : -1.f;
  const float ua = fmaf(z, uz, u0);
  float plane = uz > 0.f ? floorf(ua) + 1.f : ceilf(ua) - 1.f;
  float zc = (plane - u0) * iuz;
  for (int k = 0; k < 3 && !(zc > z); ++k) {
    plane += dir;
    zc = (plane - u0) * iuz;
  }
  return zc > z ? zc : z + fabsf(iuz);
}

// First root of the field on the ray segment [z, z + len] inside cell rc,
// given t = p + q tau (tau = height above z).  Returns tau or -1.
__device__ __forceinline__ float cell_first_root(const RayCell& rc, const float p[3], const float q[3], float len) {
  const float* a = rc.a;
  const float kx = a[1] - a[0], ky = a[2] - a[0], kz = a[4] - a[0];
  const float kxy = a[3] - a[2] - a[1] + a[0];
  const float kxz = a[5] - a[4] - a[1] + a[0];
  const float kyz = a[6] - a[4] - a[2] + a[0];
  const float kxyz = a[7] - a[6] - a[5] + a[4] - a[3] + a[2] + a[1] - a[0];
  // phi(tau) = c0 + c1 tau + c2 tau^2 + c3 tau^3 (c0 not needed)
  const float gx = kx + kxy * p[1] + kxz * p[2] + kxyz * p[1] * p[2];
  const float gy = ky + kxy * p[0] + kyz * p[2] + kxyz * p[0] * p[2];
  const float gz = kz + kxz * p[0] + kyz * p[1] + kxyz * p[0] * p[1];
  const float c1 = gx * q[0] + gy * q[1] + gz * q[2];
  const float c2 = (kxy + kxyz * p[2]) * q[0] * q[1] + (kxz + kxyz * p[1]) * q[0] * q[2] +
                   (kyz + kxyz * p[0]) * q[1] * q[2];
  const float c3 = kxyz * q[0] * q[1] * q[2];
  // critical points: 3 c3 tau^2 + 2 c2 tau + c1 = 0 (stable quadratic roots)
  float t1 = INFINITY, t2 = INFINITY;
  const float A = 3.f * c3, B = 2.f * c2, C = c1;
  if (A == 0.f) {
    if (B != 0.f) t1 = -C / B;
  } else {
    const float disc = B * B - 4.f * A * C;
    if (disc >= 0.f) {
      const float qq = -0.5f * (B + copysignf(sqrtf(disc), B));
      t1 = qq / A;
      t2 = qq != 0.f ? C / qq : INFINITY;
    }
  }
  if (t2 < t1) {
    const float t = t1;
    t1 = t2;
    t2 = t;
  }
  float pts[3] = {t1, t2, len};
  float lo = 0.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float tj = pts[j];
    if (!(tj > lo && tj <= len)) continue;  // outside the segment (or NaN)
    if (cell_tri(rc, fmaf(tj, q[0], p[0]), fmaf(tj, q[1], p[1]), fmaf(tj, q[2], p[2])) <= 0.f) {
      // phi(lo) > 0 >= phi(hi) and phi is monotone in between: Newton steps
      // on the cubic, kept inside the shrinking bracket (a step that leaves
      // it is replaced by the bracket's midpoint), until a step is below
      // 1e-6 of the segment.  A root close to one end of a long bracket can
      // send several Newton steps out of it before they converge, so the cap
      // is set by the bisections alone: 40 halvings reach 1e-12 of the segment.
      float hi = tj;
      const float c0 = cell_tri(rc, p[0], p[1], p[2]);
      float t = 0.5f * (lo + hi);
      for (int k = 0; k < 40; ++k) {
        const float f = fmaf(t, fmaf(t, fmaf(t, c3, c2), c1), c0);
        if (f == 0.f) break;
        if (f > 0.f)
          lo = t;
        else
          hi = t;
        const float d = fmaf(t, fmaf(t, 3.f * c3, 2.f * c2), c1);
        float tn = t - f / d;
        if (!(tn >= lo && tn <= hi)) tn = 0.5f * (lo + hi);  // also catches d == 0 (inf / NaN)
        const bool done = fabsf(tn - t) <= 1e-6f * len;
        t = tn;
        if (done) break;
      }
      return t;
    }
    lo = tj;
  }
  return -1.f;
}

__global__ __launch_bounds__(256) void k_depth_image(const DepthArgs a) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // workgroup b runs on XCD b % 8; all workgroups of a pad stay on one XCD,
  // which takes pad slots x, x + 8, x + 16, ... of the spatial order (each
  // object's pads cut into one run per XCD): the pad's rays share one L2 and
  // the next pad on that XCD is a spatial neighbour
  const int64_t rank = blockIdx.x >> 3;  // this workgroup's rank on its XCD
  const int64_t s = (rank / a.wg_per_pad) * 8 + (blockIdx.x & 7u);
  if (s >= a.n_inst) return;
  const int b = (int)(rank % a.wg_per_pad) * 4 + wave;  // one 8 x 8 pixel block per wavefront
  if (b >= a.blocks_per_pad) return;
  const int i = __builtin_amdgcn_readfirstlane(a.pad_order[s]);
  const int br = b / a.blocks_x, bc = b - br * a.blocks_x;
  const int r = br * 8 + (lane >> 3), c = bc * 8 + (lane & 7);
  if (r >= a.rows || c >= a.cols) return;
  const InstStatic st = a.stat[i];
  const InstXf x = a.xf[i];
  const DepthGrid g = a.grids[st.gid];
  const __amdgpu_buffer_rsrc_t rs = make_rsrc_f(g.phi, g.bytes);
  const float px = fmaf((float)c + 0.5f, a.dx, a.x0), py = fmaf((float)r + 0.5f, a.dy, a.y0);
  const float ex = a.ortho ? 0.f : px / a.cam_dist, ey = a.ortho ? 0.f : py / a.cam_dist;
  const float u0[3] = {fmaf(x.A[0], px, fmaf(x.A[1], py, x.b[0])), fmaf(x.A[3], px, fmaf(x.A[4], py, x.b[1])),
                       fmaf(x.A[6], px, fmaf(x.A[7], py, x.b[2]))};
  const float uz[3] = {fmaf(x.A[0], ex, fmaf(x.A[1], ey, x.A[2])), fmaf(x.A[3], ex, fmaf(x.A[4], ey, x.A[5])),
                       fmaf(x.A[6], ex, fmaf(x.A[7], ey, x.A[8]))};
  // one division per axis; the box clipping and the step cap multiply by it
  const float iuz[3] = {1.f / uz[0], 1.f / uz[1], 1.f / uz[2]};
  float zlo = -a.gel, zhi = 0.f;
  const int n[3] = {st.nx, st.ny, st.nz};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float n1 = (float)(n[k] - 1);
    if (uz[k] == 0.f) {
      if (!(u0[k] >= 0.f && u0[k] <= n1)) zhi = -INFINITY;
      continue;
    }
    const float za = -u0[k] * iuz[k], zb = (n1 - u0[k]) * iuz[k];
    zlo = fmaxf(zlo, fminf(za, zb));
    zhi = fminf(zhi, fmaxf(za, zb));
  }
  bool hit = false, capped = false;
  float zh = 0.f;
  if (zlo <= zhi) {
    RayCell rc;
    rc.cx = -1;
    rc.cy = -1;
    rc.cz = -1;
    const float au[3] = {fabsf(uz[0]), fabsf(uz[1]), fabsf(uz[2])};
    // at most 7 cells along any axis (1 / |uz| is infinite on an axis the ray does not move along)
    const float zcap = 7.f * fminf(fabsf(iuz[0]), fminf(fabsf(iuz[1]), fabsf(iuz[2])));
    float z = zlo;
    float u[3] = {fmaf(z, uz[0], u0[0]), fmaf(z, uz[1], u0[1]), fmaf(z, uz[2], u0[2])};
    ray_cell(st, g, rs, rc, u[0], u[1], u[2]);
    float phi = cell_tri(rc, u[0] - (float)rc.cx, u[1] - (float)rc.cy, u[2] - (float)rc.cz);
    if (phi <= 0.f) {
      hit = true;
      zh = z;
    } else {
      int it = 0;
      for (; it < kDepthMaxIter; ++it) {
        const float ze = fminf(fminf(next_plane(u0[0], uz[0], iuz[0], z), next_plane(u0[1], uz[1], iuz[1], z)),
                               next_plane(u0[2], uz[2], iuz[2], z));
        const float zend = fminf(ze, zhi);
        // the block of the current cell: the point is in it or on its boundary
        const float4 m = g.slope[((rc.cx >> 3) * g.sby + (rc.cy >> 3)) * g.sbz + (rc.cz >> 3)];
        const float bnd = fmaf(m.x, au[0], fmaf(m.y, au[1], m.z * au[2])) * 1.00002f;  // rounding margin
        const float zs = z + fminf(phi / bnd, zcap);  // phi > 0 here; bnd == 0 gives the cap
        if (zs >= zend) {  // a safe step that leaves the cell
          if (zs >= zhi) break;
          z = zs;
          u[0] = fmaf(z, uz[0], u0[0]);
          u[1] = fmaf(z, uz[1], u0[1]);
          u[2] = fmaf(z, uz[2], u0[2]);
          ray_cell(st, g, rs, rc, u[0], u[1], u[2]);
          phi = cell_tri(rc, u[0] - (float)rc.cx, u[1] - (float)rc.cy, u[2] - (float)rc.cz);
          if (phi <= 0.f) {  // only by rounding at the step's end
            hit = true;
            zh = z;
            break;
          }
          continue;
        }
        // the rest of this cell, exactly; the cell is the one holding the open segment
        const float zm = 0.5f * (z + zend);
        ray_cell(st, g, rs, rc, fmaf(zm, uz[0], u0[0]), fmaf(zm, uz[1], u0[1]), fmaf(zm, uz[2], u0[2]));
        const float p[3] = {fmaf(z, uz[0], u0[0]) - (float)rc.cx, fmaf(z, uz[1], u0[1]) - (float)rc.cy,
                            fmaf(z, uz[2], u0[2]) - (float)rc.cz};
        const float tau = cell_first_root(rc, p, uz, zend - z);
        if (tau >= 0.f) {
          hit = true;
          zh = z + tau;
          break;
        }
        if (zend >= zhi) break;
        phi = cell_tri(rc, fmaf(zend - z, uz[0], p[0]), fmaf(zend - z, uz[1], p[1]), fmaf(zend - z, uz[2], p[2]));
        z = zend;
      }
      capped = it >= kDepthMaxIter;
    }
  }
  if (capped && a.status) atomicOr(a.status, TACSL_DEV_DEPTH_CAPPED);
  __builtin_nontemporal_store((hit ? zh : 0.f) + a.cam_dist,
                              a.image + (int64_t)i * a.rows * a.cols + (int64_t)r * a.cols + c);
}

// Node values of a prepared (phi, G) grid copied into x-quad columns.
__global__ __launch_bounds__(256) void k_phi_quad(const float4* __restrict__ grid, int nx, int ny, int nz,
                                                  float* __restrict__ out) {
  const int64_t rows = (int64_t)ny * nz;
  const uint32_t sy4 = 64u * (uint32_t)nz, sq4 = sy4 * (uint32_t)((ny + 1) / 2);  // (phi, G) layout strides
  const int64_t qy = (int64_t)nz * 4, qq = qy * ny;                      // x-quad strides in floats
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const int j = (int)(row / nz), k = (int)(row % nz);
    for (int i = threadIdx.x; i < nx; i += 256) {
      const uint32_t src = (uint32_t)(i >> 1) * sq4 + (uint32_t)(j >> 1) * sy4 + (uint32_t)k * 64u +
                           (uint32_t)(j & 1) * 32u + (uint32_t)(i & 1) * 16u;
      const float v = reinterpret_cast<const float*>(reinterpret_cast<const char*>(grid) + src)[0];
      out[(int64_t)(i >> 2) * qq + (int64_t)j * qy + (int64_t)k * 4 + (i & 3)] = v;
    }
  }
}

// Slope bounds per block (layout in tacsl_internal.h), from the x-quad node
// values: first each block's own edges, then the maximum over its neighbours.
__device__ __forceinline__ float quad_at(const float* q, int i, int j, int k, int ny, int nz) {
  return q[(int64_t)(i >> 2) * 4 * ny * nz + (int64_t)4 * nz * j + 4 * k + (i & 3)];
}

__global__ __launch_bounds__(256) void k_block_slopes_raw(const float* __restrict__ q, int nx, int ny, int nz,
                                                          int sbx, int sby, int sbz, float4* __restrict__ raw) {
  const int64_t nb = (int64_t)sbx * sby * sbz;
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= nb) return;
  const int bz = (int)(b % sbz), by = (int)((b / sbz) % sby), bx = (int)(b / ((int64_t)sbz * sby));
  // nodes of the block's cells
  const int i0 = bx * kSlopeBlock, i1 = min(i0 + kSlopeBlock, nx - 1);
  const int j0 = by * kSlopeBlock, j1 = min(j0 + kSlopeBlock, ny - 1);
  const int k0 = bz * kSlopeBlock, k1 = min(k0 + kSlopeBlock, nz - 1);
  float mx = 0.f, my = 0.f, mz = 0.f;
  for (int i = i0; i <= i1; ++i)
    for (int j = j0; j <= j1; ++j)
      for (int k = k0; k <= k1; ++k) {
        const float v = quad_at(q, i, j, k, ny, nz);
        if (i < i1) mx = fmaxf(mx, fabsf(quad_at(q, i + 1, j, k, ny, nz) - v));
        if (j < j1) my = fmaxf(my, fabsf(quad_at(q, i, j + 1, k, ny, nz) - v));
        if (k < k1) mz = fmaxf(mz, fabsf(quad_at(q, i, j, k + 1, ny, nz) - v));
      }
  raw[b] = make_float4(mx, my, mz, 0.f);
}

__global__ __launch_bounds__(256) void k_block_slopes_dilate(const float4* __restrict__ raw, int sbx, int sby, int sbz,
                                                             float4* __restrict__ out) {
  const int64_t nb = (int64_t)sbx * sby * sbz;
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= nb) return;
  const int bz = (int)(b % sbz), by = (int)((b / sbz) % sby), bx = (int)(b / ((int64_t)sbz * sby));
  float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int x = max(bx - 1, 0); x <= min(bx + 1, sbx - 1); ++x)
    for (int y = max(by - 1, 0); y <= min(by + 1, sby - 1); ++y)
      for (int z = max(bz - 1, 0); z <= min(bz + 1, sbz - 1); ++z) {
        const float4 r = raw[((int64_t)x * sby + y) * sbz + z];
        m.x = fmaxf(m.x, r.x);
        m.y = fmaxf(m.y, r.y);
        m.z = fmaxf(m.z, r.z);
      }
  out[b] = m;
}

}  // namespace

hipError_t launch_phi_quad(const float4* grid, int nx, int ny, int nz, float* out, hipStream_t stream) {
  int64_t blocks = (int64_t)ny * nz;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_phi_quad, dim3((unsigned)blocks), dim3(256), 0, stream, grid, nx, ny, nz, out);
  return hipGetLastError();
}

hipError_t launch_block_slopes(const float* phi4, int nx, int ny, int nz, float4* raw, float4* out,
                               hipStream_t stream) {
  const int sbx = (int)slope_blocks(nx), sby = (int)slope_blocks(ny), sbz = (int)slope_blocks(nz);
  const int64_t nb = (int64_t)sbx * sby * sbz;
  const unsigned blocks = (unsigned)((nb + 255) / 256);
  hipLaunchKernelGGL(k_block_slopes_raw, dim3(blocks), dim3(256), 0, stream, phi4, nx, ny, nz, sbx, sby, sbz, raw);
  hipLaunchKernelGGL(k_block_slopes_dilate, dim3(blocks), dim3(256), 0, stream, raw, sbx, sby, sbz, out);
  return hipGetLastError();
}

hipError_t launch_depth_image(const DepthArgs& a, hipStream_t stream) {
  if (a.n_inst == 0 || a.blocks_per_pad == 0) return hipSuccess;
  DepthArgs b = a;
  b.wg_per_pad = (a.blocks_per_pad + 3) / 4;
  const int64_t grid = 8 * (((int64_t)a.n_inst + 7) / 8) * b.wg_per_pad;
  hipLaunchKernelGGL(k_depth_image, dim3((unsigned)grid), dim3(256), 0, stream, b);
  return hipGetLastError();
}

}  // namespace tacsl
