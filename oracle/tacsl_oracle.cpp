// FP64 CPU oracle of the tactile force field -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, step-by-step evaluation of the penalty-based tactile force
// field of Section III-C ("Normal/Shear Force-Field Computation"): for every
// tactile point of every pad it queries the object's voxelized SDF, takes the
// contact normal from finite-difference gradients of the SDF, and applies the
// force law (normal spring with depth-scaled damping, tangential force capped
// by Coulomb friction).  It exists to check the HIP implementation and is used
// only by the tests, the smoke check and the CPU-baseline leg of the
// benchmark.  It shares no code, header or helper with the HIP library.
//
// Readings of points the paper leaves open (each applied below):
//  * d is the SDF value phi, negative inside the object; n = grad(phi)
//    normalized points out of the object.  With this sign the k_d term
//    dissipates (Kelvin-Voigt law of Section III-A uses the same contact
//    distance, and the notation appendix identifies the two quantities).
//  * No contact (all outputs zero) when phi >= 0 or the tactile point is
//    outside the grid box; trilinear interpolation of node values; cell index
//    c = min(floor(u), N-2).
//  * "finite differencing" = nodal central differences (one-sided on the grid
//    faces), interpolated trilinearly with the same weights as phi.
//  * x_dot = velocity of the tactile point minus velocity of the coincident
//    object point; everything is reported in the pad frame.
//  * v_t = x_dot - (n . x_dot) n;  f_t = -k_t v_t when k_t |v_t| <= mu |f_n|
//    (stick, includes v_t = 0), else -mu |f_n| v_t / |v_t| (slip).
//  * |g| < 1e-6 (degenerate normal): n = 0 and both forces are zero.
//  * Per-pad wrench: sum of f_n + f_t and of x_p x (f_n + f_t) over the pad,
//    pad frame, torque about the pad origin.
//
// Parity pins live in tests/test_oracle_*.py.
#include <cmath>
#include <limits>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

using std::cos;
using std::fabs;
using std::sin;
using std::sqrt;

// ---------------------------------------------------------------------------
// Forward-mode dual number with a fixed number of tangent directions.
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0) { for (int i = 0; i < N; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0; }
};
template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a) { Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v / b.v; for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> Dual<N> sqrt(const Dual<N>& a) { Dual<N> r; r.v = std::sqrt(a.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / (2.0 * r.v); return r; }
template <int N> Dual<N> sin(const Dual<N>& a) { Dual<N> r; r.v = std::sin(a.v); double c = std::cos(a.v); for (int i = 0; i < N; ++i) r.d[i] = c * a.d[i]; return r; }
template <int N> Dual<N> cos(const Dual<N>& a) { Dual<N> r; r.v = std::cos(a.v); double s = -std::sin(a.v); for (int i = 0; i < N; ++i) r.d[i] = s * a.d[i]; return r; }
template <int N> Dual<N> fabs(const Dual<N>& a) { return a.v < 0 ? -a : a; }
// a^p for a > 0 and a constant exponent p
template <int N> Dual<N> powc(const Dual<N>& a, double p) {
  Dual<N> r; r.v = std::pow(a.v, p); double d = p * std::pow(a.v, p - 1.0);
  for (int i = 0; i < N; ++i) r.d[i] = d * a.d[i];
  return r;
}
inline double powc(double a, double p) { return std::pow(a, p); }

inline double val(double x) { return x; }
template <int N> inline double val(const Dual<N>& x) { return x.v; }

// ---------------------------------------------------------------------------
// Small vector / matrix helpers (generic scalar).
// ---------------------------------------------------------------------------
template <class S> struct V3 { S x, y, z; };
template <class S> V3<S> v3(S a, S b, S c) { return V3<S>{a, b, c}; }
template <class S> V3<S> add(const V3<S>& a, const V3<S>& b) { return v3<S>(a.x + b.x, a.y + b.y, a.z + b.z); }
template <class S> V3<S> sub(const V3<S>& a, const V3<S>& b) { return v3<S>(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class S> V3<S> scl(const V3<S>& a, const S& s) { return v3<S>(a.x * s, a.y * s, a.z * s); }
template <class S> S dot(const V3<S>& a, const V3<S>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S> V3<S> cross(const V3<S>& a, const V3<S>& b) {
  return v3<S>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <class S> struct M3 { S m[3][3]; };
template <class S> V3<S> mul(const M3<S>& R, const V3<S>& a) {
  return v3<S>(R.m[0][0] * a.x + R.m[0][1] * a.y + R.m[0][2] * a.z,
               R.m[1][0] * a.x + R.m[1][1] * a.y + R.m[1][2] * a.z,
               R.m[2][0] * a.x + R.m[2][1] * a.y + R.m[2][2] * a.z);
}
template <class S> V3<S> mulT(const M3<S>& R, const V3<S>& a) {  // R^T a
  return v3<S>(R.m[0][0] * a.x + R.m[1][0] * a.y + R.m[2][0] * a.z,
               R.m[0][1] * a.x + R.m[1][1] * a.y + R.m[2][1] * a.z,
               R.m[0][2] * a.x + R.m[1][2] * a.y + R.m[2][2] * a.z);
}
template <class S> M3<S> matmul(const M3<S>& A, const M3<S>& B) {
  M3<S> C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.m[i][j] = A.m[i][0] * B.m[0][j] + A.m[i][1] * B.m[1][j] + A.m[i][2] * B.m[2][j];
  return C;
}
template <class S> V3<S> lift(const V3<double>& a) { return v3<S>(S(a.x), S(a.y), S(a.z)); }
template <class S> M3<S> lift(const M3<double>& A) {
  M3<S> B;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B.m[i][j] = S(A.m[i][j]);
  return B;
}

// Rotation matrix of the normalized quaternion (w, x, y, z).
static M3<double> quat_to_R(const double* q) {
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  M3<double> R;
  R.m[0][0] = 1 - 2 * (y * y + z * z); R.m[0][1] = 2 * (x * y - w * z);     R.m[0][2] = 2 * (x * z + w * y);
  R.m[1][0] = 2 * (x * y + w * z);     R.m[1][1] = 1 - 2 * (x * x + z * z); R.m[1][2] = 2 * (y * z - w * x);
  R.m[2][0] = 2 * (x * z - w * y);     R.m[2][1] = 2 * (y * z + w * x);     R.m[2][2] = 1 - 2 * (x * x + y * y);
  return R;
}

// Rotation by the rotation vector phi (Rodrigues).  The coefficients
// sin(t)/t and (1-cos t)/t^2 are evaluated as series in t^2 for tiny angles
// so that dual numbers stay smooth at phi = 0.
template <class S> M3<S> so3_exp(const V3<S>& phi) {
  S t2 = dot(phi, phi);
  S a, b;
  if (val(t2) < 1e-8) {
    a = 1.0 - t2 / 6.0 + t2 * t2 / 120.0;
    b = 0.5 - t2 / 24.0 + t2 * t2 / 720.0;
  } else {
    S t = sqrt(t2);
    a = sin(t) / t;
    b = (1.0 - cos(t)) / t2;
  }
  // R = I + a [phi]x + b [phi]x^2
  S K[3][3] = {{S(0.0), -phi.z, phi.y}, {phi.z, S(0.0), -phi.x}, {-phi.y, phi.x, S(0.0)}};
  M3<S> R;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      S k2 = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
      R.m[i][j] = (i == j ? S(1.0) : S(0.0)) + a * K[i][j] + b * k2;
    }
  return R;
}

// ---------------------------------------------------------------------------
// Inputs (C layout shared with the Python shim).
// ---------------------------------------------------------------------------
extern "C" {
typedef struct {
  int32_t n_env, n_inst, n_tmpl, n_sdf;
  const int32_t* inst_env;    // [n_inst]
  const int32_t* inst_tmpl;   // [n_inst]
  const int32_t* env_sdf;     // [n_env]
  const int64_t* tmpl_offset; // [n_tmpl+1]
  const float* tmpl_xyz;      // [3][T_tmpl] pad frame
  const int32_t* sdf_dims;    // [n_sdf][3]
  const float* sdf_origin;    // [n_sdf][3]
  const float* sdf_spacing;   // [n_sdf]
  const int64_t* sdf_offset;  // [n_sdf]
  const float* sdf_data;      // node values, x fastest
} oracle_scene;

typedef struct {
  const double* pad_pose;       // [n_inst][7] qw qx qy qz tx ty tz
  const double* obj_pose;       // [n_env][7]
  const double* pad_twist;      // [n_inst][6] v(origin) w, world
  const double* obj_twist;      // [n_env][6]
  const double* params;         // [n_env][4] k_n k_d k_t mu
  const double* obj_pose_delta; // [n_env][6] dt dtheta (may be NULL): R_o <- Exp(dtheta) R_o, t_o <- t_o + dt
  double normal_exponent;       // p of the normal law (1: the law of Section III-C; see eval_taxel)
} oracle_state;
}

// ---------------------------------------------------------------------------
// One instance (pad) with its object, in a generic scalar type S.
// ---------------------------------------------------------------------------
template <class S> struct Instance {
  M3<double> Rp; V3<double> tp;     // pad world pose
  M3<S> Ro; V3<S> to;               // object world pose (after the optional delta)
  V3<double> vp, wp;                // pad twist
  V3<S> vo, wo;                     // object twist
  S kn, kd, kt, mu;                 // contact parameters
  double hc;                        // exponent of the penetration in the normal law (1: linear)
  // grid
  int nx, ny, nz;
  double ox, oy, oz, h;
  const float* phi;
};

struct SDFView {
  int nx, ny, nz;
  const float* phi;
  double at(int i, int j, int k) const { return (double)phi[((int64_t)k * ny + j) * nx + i]; }
  // Nodal finite-difference gradient: central inside, one-sided on the faces.
  double grad(int axis, int i, int j, int k, double h) const {
    int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    int c = axis == 0 ? i : (axis == 1 ? j : k);
    int lo = c > 0 ? c - 1 : 0;
    int hi = c < n - 1 ? c + 1 : n - 1;
    int a[3] = {i, j, k}, b[3] = {i, j, k};
    a[axis] = hi;
    b[axis] = lo;
    return (at(a[0], a[1], a[2]) - at(b[0], b[1], b[2])) / ((double)(hi - lo) * h);
  }
};

template <class S> struct TaxelOut {
  S depth;
  V3<S> n, fn, ft;
  int cell;       // linear cell index, -1 when outside the grid
  int contact;    // phi < 0
  int stick;      // 1 stick, 0 slip, -1 no friction evaluated
  int gnorm_ok;   // |g| >= 1e-6
  // the values the discrete decisions above compare (0 where not reached):
  // phi (against 0), |g| (against 1e-6), k_t |v_t| and mu |s| (against each other)
  double phi_v, gn_v, ktv_v, cap_v;
  double dcap_v;  // |d(mu |s|)/d phi|: how far an error in phi moves the friction cap
};

template <class S>
static TaxelOut<S> eval_taxel(const Instance<S>& I, const V3<double>& xp) {
  TaxelOut<S> o;
  o.depth = S(0.0);
  o.n = o.fn = o.ft = v3<S>(S(0.0), S(0.0), S(0.0));
  o.cell = -1; o.contact = 0; o.stick = -1; o.gnorm_ok = 0;
  o.phi_v = o.gn_v = o.ktv_v = o.cap_v = o.dcap_v = std::numeric_limits<double>::quiet_NaN();

  // (1) taxel to world and to object frame.
  V3<double> xw = add(mul(I.Rp, xp), I.tp);
  V3<S> xo = mulT(I.Ro, sub(lift<S>(xw), I.to));
  // (2) grid coordinates; outside the node box means no contact.
  S u[3] = {(xo.x - I.ox) / I.h, (xo.y - I.oy) / I.h, (xo.z - I.oz) / I.h};
  int n[3] = {I.nx, I.ny, I.nz};
  for (int a = 0; a < 3; ++a)
    if (!(val(u[a]) >= 0.0 && val(u[a]) <= (double)(n[a] - 1))) return o;
  // (3) cell and local coordinates.
  int c[3];
  S t[3];
  for (int a = 0; a < 3; ++a) {
    int f = (int)std::floor(val(u[a]));
    c[a] = f < n[a] - 2 ? f : n[a] - 2;
    t[a] = u[a] - (double)c[a];
  }
  o.cell = (c[2] * I.ny + c[1]) * I.nx + c[0];
  SDFView g{I.nx, I.ny, I.nz, I.phi};
  // (4) trilinear value and (6) trilinear nodal gradient.
  S phi(0.0);
  S gx(0.0), gy(0.0), gz(0.0);
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        S w = (dx ? t[0] : 1.0 - t[0]) * (dy ? t[1] : 1.0 - t[1]) * (dz ? t[2] : 1.0 - t[2]);
        int i = c[0] + dx, j = c[1] + dy, k = c[2] + dz;
        phi = phi + w * g.at(i, j, k);
        gx = gx + w * g.grad(0, i, j, k, I.h);
        gy = gy + w * g.grad(1, i, j, k, I.h);
        gz = gz + w * g.grad(2, i, j, k, I.h);
      }
  o.phi_v = val(phi);
  // (5) no contact for phi >= 0.
  if (!(val(phi) < 0.0)) return o;
  o.contact = 1;
  o.depth = -phi;
  S gn = sqrt(gx * gx + gy * gy + gz * gz);
  o.gn_v = val(gn);
  if (!(val(gn) >= 1e-6)) return o;  // degenerate normal: no force
  o.gnorm_ok = 1;
  V3<S> no = v3<S>(gx / gn, gy / gn, gz / gn);
  // (7) normal and relative velocity in the pad frame.
  V3<S> nw = mul(I.Ro, no);
  M3<S> Rp = lift<S>(I.Rp);
  V3<S> n_p = mulT(Rp, nw);
  V3<S> vpad = add(lift<S>(I.vp), lift<S>(cross(I.wp, sub(xw, I.tp))));
  V3<S> vobj = add(I.vo, cross(I.wo, sub(lift<S>(xw), I.to)));
  V3<S> xdot = mulT(Rp, sub(vpad, vobj));
  // (8) normal force f_n = (-k_n + k_d d_dot) d n with d = phi.  With an
  // exponent p != 1 the penetration -phi enters as (-phi)^p: the nonlinear
  // (Hunt-Crossley) variant named in Section VII, damping still scaled by
  // the same power of the penetration.
  S ddot = dot(n_p, xdot);
  S dpow = I.hc == 1.0 ? phi : -powc(-phi, I.hc);
  S s = (-I.kn + I.kd * ddot) * dpow;
  o.n = n_p;
  o.fn = scl(n_p, s);
  // (9) friction: f_t = -v_t/|v_t| min(k_t |v_t|, mu |f_n|).
  V3<S> vt = sub(xdot, scl(n_p, ddot));
  S vtn = sqrt(dot(vt, vt));
  S cap = I.mu * fabs(s);
  o.ktv_v = val(I.kt) * val(vtn);
  o.cap_v = val(cap);
  {
    const double dp = I.hc == 1.0 ? 1.0 : I.hc * std::pow(-val(phi), I.hc - 1.0);
    o.dcap_v = val(I.mu) * std::fabs(-val(I.kn) + val(I.kd) * val(ddot)) * dp;
  }
  if (val(I.kt) * val(vtn) <= val(cap)) {
    o.stick = 1;
    o.ft = scl(vt, -I.kt);
  } else {
    o.stick = 0;
    o.ft = scl(vt, -cap / vtn);
  }
  return o;
}

template <class S>
static void setup_instance(const oracle_scene& sc, const oracle_state& st, int i, Instance<S>& I,
                           const V3<S>* dt = nullptr, const V3<S>* dth = nullptr) {
  int e = sc.inst_env[i];
  int sd = sc.env_sdf[e];
  I.Rp = quat_to_R(st.pad_pose + 7 * (int64_t)i);
  I.tp = v3<double>(st.pad_pose[7 * (int64_t)i + 4], st.pad_pose[7 * (int64_t)i + 5], st.pad_pose[7 * (int64_t)i + 6]);
  M3<double> Ro = quat_to_R(st.obj_pose + 7 * (int64_t)e);
  V3<S> to = v3<S>(S(st.obj_pose[7 * (int64_t)e + 4]), S(st.obj_pose[7 * (int64_t)e + 5]), S(st.obj_pose[7 * (int64_t)e + 6]));
  V3<S> ddt = v3<S>(S(0.0), S(0.0), S(0.0)), ddth = ddt;
  if (st.obj_pose_delta) {
    const double* d = st.obj_pose_delta + 6 * (int64_t)e;
    ddt = v3<S>(S(d[0]), S(d[1]), S(d[2]));
    ddth = v3<S>(S(d[3]), S(d[4]), S(d[5]));
  }
  if (dt) ddt = add(ddt, *dt);
  if (dth) ddth = add(ddth, *dth);
  I.Ro = matmul(so3_exp(ddth), lift<S>(Ro));
  I.to = add(to, ddt);
  const double* pt = st.pad_twist + 6 * (int64_t)i;
  I.vp = v3<double>(pt[0], pt[1], pt[2]);
  I.wp = v3<double>(pt[3], pt[4], pt[5]);
  const double* ot = st.obj_twist + 6 * (int64_t)e;
  I.vo = v3<S>(S(ot[0]), S(ot[1]), S(ot[2]));
  I.wo = v3<S>(S(ot[3]), S(ot[4]), S(ot[5]));
  const double* p = st.params + 4 * (int64_t)e;
  I.kn = S(p[0]); I.kd = S(p[1]); I.kt = S(p[2]); I.mu = S(p[3]);
  I.hc = st.normal_exponent > 0.0 ? st.normal_exponent : 1.0;
  I.nx = sc.sdf_dims[3 * sd]; I.ny = sc.sdf_dims[3 * sd + 1]; I.nz = sc.sdf_dims[3 * sd + 2];
  I.ox = sc.sdf_origin[3 * sd]; I.oy = sc.sdf_origin[3 * sd + 1]; I.oz = sc.sdf_origin[3 * sd + 2];
  I.h = sc.sdf_spacing[sd];
  I.phi = sc.sdf_data + sc.sdf_offset[sd];
}

static int64_t tmpl_count(const oracle_scene& sc, int i) {
  int p = sc.inst_tmpl[i];
  return sc.tmpl_offset[p + 1] - sc.tmpl_offset[p];
}
static V3<double> tmpl_point(const oracle_scene& sc, int i, int64_t k) {
  int p = sc.inst_tmpl[i];
  int64_t T = sc.tmpl_offset[sc.n_tmpl];
  int64_t j = sc.tmpl_offset[p] + k;
  return v3<double>(sc.tmpl_xyz[j], sc.tmpl_xyz[T + j], sc.tmpl_xyz[2 * T + j]);
}

extern "C" {

// Global taxel index base of each instance: instance-major prefix sums of the
// taxel counts of the instances' templates.  out[n_inst+1].
int oracle_offsets(const oracle_scene* sc, int64_t* out) {
  out[0] = 0;
  for (int i = 0; i < sc->n_inst; ++i) out[i + 1] = out[i] + tmpl_count(*sc, i);
  return 0;
}

// Forward field for the selected instances.  Outputs are packed in selection
// order: depth[Ts], normal/fn/ft [3][Ts] (pad frame), wrench [n_sel][6]
// (force, torque about the pad origin, pad frame), and optionally per-taxel
// signatures sig[Ts][4] = (cell, contact, stick, gnorm_ok).
int oracle_force_field(const oracle_scene* sc, const oracle_state* st, int n_sel, const int32_t* sel,
                       double* depth, double* normal, double* fn, double* ft, double* wrench,
                       int32_t* sig, int nthreads) {
  std::vector<int64_t> base(n_sel + 1, 0);
  for (int s = 0; s < n_sel; ++s) base[s + 1] = base[s] + tmpl_count(*sc, sel[s]);
  const int64_t Ts = base[n_sel];
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < n_sel; ++s) {
    int i = sel[s];
    Instance<double> I;
    setup_instance<double>(*sc, *st, i, I);
    double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
    int64_t cnt = tmpl_count(*sc, i);
    for (int64_t k = 0; k < cnt; ++k) {
      V3<double> xp = tmpl_point(*sc, i, k);
      TaxelOut<double> o = eval_taxel(I, xp);
      int64_t j = base[s] + k;
      depth[j] = o.depth;
      normal[j] = o.n.x; normal[Ts + j] = o.n.y; normal[2 * Ts + j] = o.n.z;
      fn[j] = o.fn.x; fn[Ts + j] = o.fn.y; fn[2 * Ts + j] = o.fn.z;
      ft[j] = o.ft.x; ft[Ts + j] = o.ft.y; ft[2 * Ts + j] = o.ft.z;
      V3<double> f = add(o.fn, o.ft);
      V3<double> tq = cross(xp, f);
      F[0] += f.x; F[1] += f.y; F[2] += f.z;
      T[0] += tq.x; T[1] += tq.y; T[2] += tq.z;
      if (sig) {
        sig[4 * j] = o.cell; sig[4 * j + 1] = o.contact; sig[4 * j + 2] = o.stick; sig[4 * j + 3] = o.gnorm_ok;
      }
    }
    for (int a = 0; a < 3; ++a) { wrench[6 * s + a] = F[a]; wrench[6 * s + 3 + a] = T[a]; }
  }
  return 0;
}

// Scalar loss per selected environment, L_e = sum over the taxels of the
// environment's pads of a . f_n + b . f_t, and its gradient by forward-mode
// dual numbers in 16 directions: object pose perturbation (dt[3], dtheta[3];
// R_o <- Exp(dtheta) R_o, t_o <- t_o + dt, world frame, at the state's
// obj_pose_delta), object twist (v[3], w[3], world), params (k_n,k_d,k_t,mu).
// Weights wa/wb are [3][T] indexed by the global taxel index; mask (may be
// NULL) zeroes a taxel's contribution when 0.  gabs (may be NULL) receives,
// per environment and direction, the sum over taxels of the absolute value
// of each taxel's contribution to the gradient (the scale of a sum that
// cancels).
int oracle_grad(const oracle_scene* sc, const oracle_state* st, const double* wa, const double* wb,
                const uint8_t* mask, int n_sel_env, const int32_t* sel_env, double* loss, double* grad,
                double* gabs, int nthreads) {
  typedef Dual<16> D;
  std::vector<int64_t> off(sc->n_inst + 1);
  oracle_offsets(sc, off.data());
  const int64_t T = off[sc->n_inst];
  // instances of each env in ascending order
  std::vector<std::vector<int>> env_inst(sc->n_env);
  for (int i = 0; i < sc->n_inst; ++i) env_inst[sc->inst_env[i]].push_back(i);
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < n_sel_env; ++s) {
    int e = sel_env[s];
    D acc(0.0);
    double aabs[16] = {0};
    for (int i : env_inst[e]) {
      V3<D> dt, dth;
      D* comps[6] = {&dt.x, &dt.y, &dt.z, &dth.x, &dth.y, &dth.z};
      for (int a = 0; a < 6; ++a) { *comps[a] = D(0.0); comps[a]->d[a] = 1.0; }
      Instance<D> I;
      setup_instance<D>(*sc, *st, i, I, &dt, &dth);
      D* tw[6] = {&I.vo.x, &I.vo.y, &I.vo.z, &I.wo.x, &I.wo.y, &I.wo.z};
      for (int a = 0; a < 6; ++a) tw[a]->d[6 + a] = 1.0;
      I.kn.d[12] = 1.0; I.kd.d[13] = 1.0; I.kt.d[14] = 1.0; I.mu.d[15] = 1.0;
      int64_t cnt = tmpl_count(*sc, i);
      for (int64_t k = 0; k < cnt; ++k) {
        int64_t j = off[i] + k;
        if (mask && !mask[j]) continue;
        TaxelOut<D> o = eval_taxel(I, tmpl_point(*sc, i, k));
        D l = o.fn.x * wa[j] + o.fn.y * wa[T + j] + o.fn.z * wa[2 * T + j] +
              o.ft.x * wb[j] + o.ft.y * wb[T + j] + o.ft.z * wb[2 * T + j];
        acc = acc + l;
        for (int a = 0; a < 16; ++a) aabs[a] += std::fabs(l.d[a]);
      }
    }
    loss[s] = acc.v;
    for (int a = 0; a < 16; ++a) grad[16 * s + a] = acc.d[a];
    if (gabs)
      for (int a = 0; a < 16; ++a) gabs[16 * s + a] = aabs[a];
  }
  return 0;
}

// The same loss in plain FP64 (for central finite differences).
int oracle_loss(const oracle_scene* sc, const oracle_state* st, const double* wa, const double* wb,
                const uint8_t* mask, int n_sel_env, const int32_t* sel_env, double* loss, int nthreads) {
  std::vector<int64_t> off(sc->n_inst + 1);
  oracle_offsets(sc, off.data());
  const int64_t T = off[sc->n_inst];
  std::vector<std::vector<int>> env_inst(sc->n_env);
  for (int i = 0; i < sc->n_inst; ++i) env_inst[sc->inst_env[i]].push_back(i);
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < n_sel_env; ++s) {
    int e = sel_env[s];
    double acc = 0.0;
    for (int i : env_inst[e]) {
      Instance<double> I;
      setup_instance<double>(*sc, *st, i, I);
      int64_t cnt = tmpl_count(*sc, i);
      for (int64_t k = 0; k < cnt; ++k) {
        int64_t j = off[i] + k;
        if (mask && !mask[j]) continue;
        TaxelOut<double> o = eval_taxel(I, tmpl_point(*sc, i, k));
        acc += o.fn.x * wa[j] + o.fn.y * wa[T + j] + o.fn.z * wa[2 * T + j] +
               o.ft.x * wb[j] + o.ft.y * wb[T + j] + o.ft.z * wb[2 * T + j];
      }
    }
    loss[s] = acc;
  }
  return 0;
}

// Per-taxel discrete signature (cell, contact, stick, gnorm_ok) for every
// taxel of the scene in global order; sig[T][4].
int oracle_signature(const oracle_scene* sc, const oracle_state* st, int32_t* sig, int nthreads) {
  std::vector<int64_t> off(sc->n_inst + 1);
  oracle_offsets(sc, off.data());
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < sc->n_inst; ++i) {
    Instance<double> I;
    setup_instance<double>(*sc, *st, i, I);
    int64_t cnt = tmpl_count(*sc, i);
    for (int64_t k = 0; k < cnt; ++k) {
      TaxelOut<double> o = eval_taxel(I, tmpl_point(*sc, i, k));
      int64_t j = off[i] + k;
      sig[4 * j] = o.cell; sig[4 * j + 1] = o.contact; sig[4 * j + 2] = o.stick; sig[4 * j + 3] = o.gnorm_ok;
    }
  }
  return 0;
}

// Per-taxel values behind the discrete decisions of the force law, for every
// taxel of the scene in global order: m[T][5] = (phi, |g|, k_t |v_t|, mu |s|,
// |d(mu |s|)/d phi|) (NaN where the step is not reached).  Test infrastructure: tells which
// decisions lie so close to their threshold that FP32 and FP64 may take them
// differently (Section III-C: contact where the SDF is negative; friction
// min(k_t |v_t|, mu |f_n|)).
int oracle_decision_values(const oracle_scene* sc, const oracle_state* st, double* m, int nthreads) {
  std::vector<int64_t> off(sc->n_inst + 1);
  oracle_offsets(sc, off.data());
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < sc->n_inst; ++i) {
    Instance<double> I;
    setup_instance<double>(*sc, *st, i, I);
    int64_t cnt = tmpl_count(*sc, i);
    for (int64_t k = 0; k < cnt; ++k) {
      TaxelOut<double> o = eval_taxel(I, tmpl_point(*sc, i, k));
      int64_t j = off[i] + k;
      m[5 * j] = o.phi_v; m[5 * j + 1] = o.gn_v; m[5 * j + 2] = o.ktv_v; m[5 * j + 3] = o.cap_v;
      m[5 * j + 4] = o.dcap_v;
    }
  }
  return 0;
}

// Number of distinct SDF nodes read by the selected instances: the 8 corner
// nodes of every in-grid taxel, plus, for taxels in contact, the neighbours
// the central differences of those corners use.  Counted per (grid, node).
int64_t oracle_footprint(const oracle_scene* sc, const oracle_state* st, int n_sel, const int32_t* sel) {
  int64_t total_nodes = 0;
  std::vector<int64_t> sdf_base(sc->n_sdf);
  for (int g = 0; g < sc->n_sdf; ++g) {
    sdf_base[g] = total_nodes;
    total_nodes += (int64_t)sc->sdf_dims[3 * g] * sc->sdf_dims[3 * g + 1] * sc->sdf_dims[3 * g + 2];
  }
  std::vector<uint8_t> seen((size_t)total_nodes, 0);
  for (int s = 0; s < n_sel; ++s) {
    int i = sel[s];
    int sd = sc->env_sdf[sc->inst_env[i]];
    Instance<double> I;
    setup_instance<double>(*sc, *st, i, I);
    int64_t cnt = tmpl_count(*sc, i);
    int n[3] = {I.nx, I.ny, I.nz};
    for (int64_t k = 0; k < cnt; ++k) {
      TaxelOut<double> o = eval_taxel(I, tmpl_point(*sc, i, k));
      if (o.cell < 0) continue;
      int c[3] = {o.cell % I.nx, (o.cell / I.nx) % I.ny, o.cell / (I.nx * I.ny)};
      for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            int p[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
            seen[sdf_base[sd] + ((int64_t)p[2] * I.ny + p[1]) * I.nx + p[0]] = 1;
            if (!o.contact) continue;
            for (int a = 0; a < 3; ++a)
              for (int sgn = -1; sgn <= 1; sgn += 2) {
                int q[3] = {p[0], p[1], p[2]};
                q[a] += sgn;
                if (q[a] < 0 || q[a] >= n[a]) continue;
                seen[sdf_base[sd] + ((int64_t)q[2] * I.ny + q[1]) * I.nx + q[0]] = 1;
              }
          }
    }
  }
  int64_t count = 0;
  for (size_t j = 0; j < seen.size(); ++j) count += seen[j];
  return count;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Tactile depth image (Section III-B): a camera inside the sensor, behind the
// gel, sees the indenting object.  Pixel (r, c) looks through the pad-plane
// point P = (x0 + (c + 1/2) dx, y0 + (r + 1/2) dy, 0) (pad frame, +z towards
// the object).  The ray is parametrized by its pad-frame height z: for a
// pinhole at (0, 0, -D) its point at height z is P (z + D) / D in x, y;
// for an orthographic camera it is (P_x, P_y, z).  The gel occupies
// z in [-gel, 0].  The pixel reads the z-distance from the camera plane
// z = -D to the first point of the ray inside the gel where the object's
// (trilinear) SDF is <= 0, or to the gel surface z = 0 when there is none.
// Outside the grid's node box the object is absent.
//
// Along the ray the grid coordinates are affine in z, so inside one cell the
// trilinear field is a cubic in z.  The ray is walked cell by cell over the
// part of [-gel, 0] inside the node box; in each cell the cubic is sampled
// at 64 points and the first sign change is bisected to machine precision.
// slope[] receives d(phi)/dz at the hit (0 without a hit; its size tells how
// well the hit is conditioned), phimin[] the smallest sampled phi on the
// searched segment (how close a ray without a hit came to the surface).
// ---------------------------------------------------------------------------
extern "C" {
typedef struct {
  int32_t rows, cols;
  int32_t ortho;         // 1: rays parallel to +z; 0: pinhole at (0, 0, -cam_dist)
  double x0, y0, dx, dy; // pixel grid on the pad plane (pad frame, metres)
  double cam_dist;       // camera plane z = -cam_dist (>= gel)
  double gel;            // gel thickness
} oracle_camera;
}

struct RayCell {
  double a[8];  // corner values, index dx + 2 dy + 4 dz
};

static double tri_at(const RayCell& rc, double tx, double ty, double tz) {
  const double* a = rc.a;
  double x00 = a[0] + (a[1] - a[0]) * tx, x10 = a[2] + (a[3] - a[2]) * tx;
  double x01 = a[4] + (a[5] - a[4]) * tx, x11 = a[6] + (a[7] - a[6]) * tx;
  double y0 = x00 + (x10 - x00) * ty, y1 = x01 + (x11 - x01) * ty;
  return y0 + (y1 - y0) * tz;
}

extern "C" int oracle_depth_image(const oracle_scene* sc, const oracle_state* st, const oracle_camera* cam, int n_sel,
                                  const int32_t* sel, double* image, double* slope, double* phimin, int nthreads) {
  const int64_t npx = (int64_t)cam->rows * cam->cols;
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int s = 0; s < n_sel; ++s) {
    Instance<double> I;
    setup_instance<double>(*sc, *st, sel[s], I);
    SDFView g{I.nx, I.ny, I.nz, I.phi};
    const int n[3] = {I.nx, I.ny, I.nz};
    const double D = cam->cam_dist;
    for (int r = 0; r < cam->rows; ++r)
      for (int c = 0; c < cam->cols; ++c) {
        const int64_t q = (int64_t)s * npx + (int64_t)r * cam->cols + c;
        const double px = cam->x0 + (c + 0.5) * cam->dx, py = cam->y0 + (r + 0.5) * cam->dy;
        // ray point at height z (pad frame) and its grid coordinates u(z) = u0 + z uz
        V3<double> X0 = v3<double>(px, py, 0.0);
        V3<double> Xz = cam->ortho ? v3<double>(0.0, 0.0, 1.0) : v3<double>(px / D, py / D, 1.0);
        V3<double> O0 = mulT(I.Ro, sub(add(mul(I.Rp, X0), I.tp), I.to));
        V3<double> Oz = mulT(I.Ro, mul(I.Rp, Xz));
        double u0[3] = {(O0.x - I.ox) / I.h, (O0.y - I.oy) / I.h, (O0.z - I.oz) / I.h};
        double uz[3] = {Oz.x / I.h, Oz.y / I.h, Oz.z / I.h};
        double zlo = -cam->gel, zhi = 0.0;
        for (int a = 0; a < 3; ++a) {
          if (uz[a] == 0.0) {
            if (!(u0[a] >= 0.0 && u0[a] <= n[a] - 1)) zlo = 1.0, zhi = 0.0;
            continue;
          }
          double za = (0.0 - u0[a]) / uz[a], zb = (n[a] - 1 - u0[a]) / uz[a];
          if (za > zb) std::swap(za, zb);
          zlo = std::max(zlo, za);
          zhi = std::min(zhi, zb);
        }
        double zhit = 0.0, sl = 0.0, pmin = INFINITY;
        bool hit = false;
        double z = zlo;
        while (!hit && z < zhi) {
          // end of the current cell along the ray: the next integer plane crossed
          double znext = zhi;
          for (int a = 0; a < 3; ++a) {
            if (uz[a] == 0.0) continue;
            const double ua = u0[a] + z * uz[a];
            const double dir = uz[a] > 0 ? 1.0 : -1.0;
            double plane = uz[a] > 0 ? std::floor(ua) + 1.0 : std::ceil(ua) - 1.0;
            double zc = (plane - u0[a]) / uz[a];
            // a start that rounds onto (or just before) a plane: take the plane after it
            while (!(zc > z)) {
              plane += dir;
              zc = (plane - u0[a]) / uz[a];
            }
            if (zc < znext) znext = zc;
          }
          const double zm = 0.5 * (z + znext);
          int cc[3];
          for (int a = 0; a < 3; ++a) {
            int f = (int)std::floor(u0[a] + zm * uz[a]);
            cc[a] = std::min(std::max(f, 0), n[a] - 2);
          }
          RayCell rc;
          for (int k = 0; k < 8; ++k) rc.a[k] = g.at(cc[0] + (k & 1), cc[1] + ((k >> 1) & 1), cc[2] + (k >> 2));
          auto phi_at = [&](double zz) {
            return tri_at(rc, u0[0] + zz * uz[0] - cc[0], u0[1] + zz * uz[1] - cc[1], u0[2] + zz * uz[2] - cc[2]);
          };
          const int K = 64;
          double zp = z, fp = phi_at(z);
          pmin = std::min(pmin, fp);
          if (fp <= 0.0) {
            hit = true;
            zhit = z;
          }
          for (int k = 1; k <= K && !hit; ++k) {
            double zk = z + (znext - z) * k / K;
            double fk = phi_at(zk);
            pmin = std::min(pmin, fk);
            if (fk <= 0.0) {
              double lo = zp, hi = zk;  // phi(lo) > 0 >= phi(hi)
              for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (phi_at(mid) <= 0.0) hi = mid; else lo = mid;
              }
              hit = true;
              zhit = hi;
            }
            zp = zk;
            fp = fk;
          }
          if (hit) {
            const double e = 1e-9 * I.h;
            sl = (phi_at(std::min(zhit + e, znext)) - phi_at(std::max(zhit - e, z))) /
                 (std::min(zhit + e, znext) - std::max(zhit - e, z));
          }
          z = znext;
        }
        image[q] = (hit ? zhit : 0.0) + D;
        if (slope) slope[q] = hit ? sl : 0.0;
        if (phimin) phimin[q] = std::isfinite(pmin) ? pmin : 0.0;
      }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Implicit soft-contact impulse (Section III-A, "Constraint Solution").
// The Kelvin-Voigt contact force is applied as an implicit spring: the
// impulse over a step satisfies the force law at the END of the step,
//   lambda = dt max(-kappa eps+ - c epsdot+, 0),
//   epsdot+ = epsdot + lambda / m,  eps+ = eps + dt epsdot+,
// whose solution is lambda = max(0, (-dt kappa eps - alpha epsdot) / (1 + alpha/m))
// with alpha = dt (dt kappa + c).  Per contact, FP64; inv_mass = 1/m (0 for
// an immovable body); kappa, c per environment.
// ---------------------------------------------------------------------------
extern "C" int oracle_contact_impulse(int64_t n, const double* eps, const double* epsdot, const double* inv_mass,
                                      const int32_t* env, const double* kc, double dt, double* lambda, double* dv) {
  for (int64_t k = 0; k < n; ++k) {
    const int e = env ? env[k] : 0;
    const double kappa = kc[2 * e], c = kc[2 * e + 1];
    const double alpha = dt * (dt * kappa + c);
    double l = (-dt * kappa * eps[k] - alpha * epsdot[k]) / (1.0 + alpha * inv_mass[k]);
    if (!(l > 0.0)) l = 0.0;
    lambda[k] = l;
    if (dv) dv[k] = l * inv_mass[k];
  }
  return 0;
}
