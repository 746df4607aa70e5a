// Plain FP64 CPU oracle for constant-memory differentiable light tracing.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code with
// the HIP path; both read the same seeded scene arrays and nothing else.
//
// What it computes (plain definitions, no blocking or fusion):
//  * the light-tracing image: every light path x0..xk from the emitter, with a
//    sensor connection at every non-specular vertex i >= 1, each contribution
//    L_i = W_e f_i G V splatted through a tent reconstruction filter
//    (Sec. 3.1, Eq. 1-2; splat of Eq. 20);
//  * the gradient of the loss by *generic taped reverse-mode AD* of the whole
//    per-path computation (the naive AD baseline of Sec. 3.2), with the
//    image adjoint dI supplied by the caller: d/dtheta <dI, I(theta)>;
//  * the ResLRB estimator's gradient: the same tape seeded only at the
//    reservoir-selected connection R with the weight Omega_k / omega_R held
//    fixed (Sec. 4.2, Eq. 8-11);
//  * the camera side of the bidirectional combination the paper names as
//    its next step (Sec. 7): camera samples traced by a path tracer with
//    next-event estimation at Lambertian and rough-conductor vertices and
//    emission counted after specular bounces, either restricted to samples
//    whose first vertex is specular (the paths no light-path connection can
//    reach: light paths plus these samples partition the measurement of
//    Eq. 1) or unrestricted (a full path tracer, the tests' reference); and
//    its detached gradient by taped reverse-mode AD per sample;
//  * per-path decision signatures (hit primitive, texel, validity, lobe, R)
//    so that FP32/FP64 decision flips can be told apart from arithmetic
//    differences.
// Parity pins live in the test suite (closed forms, invariants, finite
// differences, reservoir pmf).
//
// Scene conventions (shared *specification*, implemented separately here):
//  - RNG: Philox-4x32-10 (Salmon et al., SC'11), key = 64-bit seed,
//    counter = (path, vertex, block, 0); u = (x >> 8) * 2^-24.
//    Vertex 0: u0,u1 emitter position, u2,u3 emitted direction.
//    Vertex j>=1: u0,u1 diffuse direction, u2 Fresnel lobe, u3 reservoir.
//    Camera sample s: block 2 at vertex 0 (u0,u1 tent-filtered film offset)
//    and at vertex j (u0,u1 scatter direction, u2 Fresnel lobe), block 3 at
//    vertex j (u0,u1 point on the quad emitter for next-event estimation);
//    its pixel is s mod (W H).
//  - Only the primitive choice uses the offset ray origin; the differentiable
//    hit point is recomputed from the true origin and the hit triangle's plane.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

// ----------------------------------------------------------------- Philox
struct U4 { uint32_t x[4]; };

U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * c.x[0];
    uint64_t p1 = (uint64_t)M1 * c.x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    U4 n;
    n.x[0] = hi1 ^ c.x[1] ^ k0;
    n.x[1] = lo1;
    n.x[2] = hi0 ^ c.x[3] ^ k1;
    n.x[3] = lo0;
    c = n;
  }
  return c;
}

struct Uniform4 { double u[4]; };

Uniform4 rng4(uint64_t seed, uint32_t path, uint32_t vertex, uint32_t block) {
  U4 c{{path, vertex, block, 0u}};
  U4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  Uniform4 o;
  for (int i = 0; i < 4; ++i) o.u[i] = (double)(r.x[i] >> 8) * (1.0 / 16777216.0);
  return o;
}

uint32_t fnv1a(uint32_t h, uint32_t w) {
  for (int b = 0; b < 4; ++b) { h ^= (w >> (8 * b)) & 0xFFu; h *= 0x01000193u; }
  return h;
}

// ----------------------------------------------------------------- tape AD
struct Tape {
  std::vector<int> a, b;
  std::vector<double> da, db;
  std::vector<std::pair<int, long>> leaves;  // (node, parameter slot)
  void clear() { a.clear(); b.clear(); da.clear(); db.clear(); leaves.clear(); }
  int push(int ia, double pa, int ib, double pb) {
    a.push_back(ia); da.push_back(pa); b.push_back(ib); db.push_back(pb);
    return (int)a.size() - 1;
  }
};
thread_local Tape* g_tape = nullptr;

struct V {
  double v; int i;
  V() : v(0.0), i(-1) {}
  V(double x) : v(x), i(-1) {}
  V(double x, int idx) : v(x), i(idx) {}
};

inline V node(double v, const V& a, double da) {
  if (a.i < 0) return V(v);
  return V(v, g_tape->push(a.i, da, -1, 0.0));
}
inline V node(double v, const V& a, double da, const V& b, double db) {
  if (a.i < 0 && b.i < 0) return V(v);
  return V(v, g_tape->push(a.i, da, b.i, db));
}
V leaf(double v, long slot) {
  int id = g_tape->push(-1, 0.0, -1, 0.0);
  g_tape->leaves.push_back({id, slot});
  return V(v, id);
}

inline V operator+(const V& a, const V& b) { return node(a.v + b.v, a, 1.0, b, 1.0); }
inline V operator-(const V& a, const V& b) { return node(a.v - b.v, a, 1.0, b, -1.0); }
inline V operator*(const V& a, const V& b) { return node(a.v * b.v, a, b.v, b, a.v); }
inline V operator/(const V& a, const V& b) {
  double q = a.v / b.v;
  return node(q, a, 1.0 / b.v, b, -q / b.v);
}
inline V operator-(const V& a) { return node(-a.v, a, -1.0); }
inline V vsqrt(const V& a) { double s = std::sqrt(a.v); return node(s, a, 0.5 / s); }
inline V vabs(const V& a) { return node(std::fabs(a.v), a, a.v >= 0 ? 1.0 : -1.0); }

struct V3 { V x, y, z; };
inline V3 operator+(const V3& a, const V3& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(const V3& a, const V3& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(const V3& a, const V& s) { return {a.x * s, a.y * s, a.z * s}; }
inline V dot(const V3& a, const V3& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(const V3& a, const V3& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline V3 normalize(const V3& a) { V l = vsqrt(dot(a, a)); return {a.x / l, a.y / l, a.z / l}; }

struct D3 { double x, y, z; };
inline D3 val(const V3& a) { return {a.x.v, a.y.v, a.z.v}; }
inline D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline D3 operator*(D3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline D3 cross(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline D3 normalize(D3 a) { double l = std::sqrt(dot(a, a)); return {a.x / l, a.y / l, a.z / l}; }
inline V3 cst(D3 a) { return {V(a.x), V(a.y), V(a.z)}; }

// Orthonormal basis from a unit normal (Duff et al., "Building an
// Orthonormal Basis, Revisited", JCGT 2017).
void onb(D3 n, D3& b1, D3& b2) {
  double sign = std::copysign(1.0, n.z);
  double a = -1.0 / (sign + n.z);
  double b = n.x * n.y * a;
  b1 = {1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x};
  b2 = {b, sign + n.y * n.y * a, -n.y};
}

void onbv(const V3& n, V3& b1, V3& b2) {
  double sign = std::copysign(1.0, n.z.v);
  V a = V(-1.0) / (V(sign) + n.z);
  V b = n.x * n.y * a;
  b1 = {V(1.0) + V(sign) * n.x * n.x * a, V(sign) * b, -(V(sign) * n.x)};
  b2 = {b, V(sign) + n.y * n.y * a, -n.y};
}

}  // namespace

// ----------------------------------------------------------------- C API
extern "C" {

enum { ORA_ABSORBER = 0, ORA_LAMBERT = 1, ORA_DIELECTRIC = 2, ORA_CONDUCTOR = 3 };
enum { ORA_EMIT_QUAD = 0, ORA_EMIT_POINT = 1, ORA_EMIT_DIRECTIONAL = 2 };
enum { ORA_F_ATTACHED = 1, ORA_F_SPLAT_SELECTED = 2 };
enum { ORA_MODE_NAIVE = 0, ORA_MODE_RESLRB = 1 };

typedef struct {
  int32_t n_tris; const double* tri_v; const double* tri_uv; const int32_t* tri_mat;
  int32_t n_mats; const int32_t* mat_type; const int32_t* mat_tex; const double* mat_ior;
  int32_t n_tex, tex_res;
  int32_t em_type; double em_o[3], em_e1[3], em_e2[3];
  double cam_pos[3], cam_target[3], cam_up[3], cam_fov_deg; int32_t width, height;
  int32_t hf_G; double hf_x0, hf_z0, hf_dx, hf_base; int32_t hf_mat;
  int32_t em_tex_res;   // > 0: the emitter's radiance is an em_tex_res^2 RGB texture over its quad
} ora_scene;

typedef struct {
  uint64_t seed; int64_t n_paths; int32_t max_depth; int32_t flags; int32_t n_threads;
  const uint32_t* path_list; int64_t n_list;   // NULL: all paths [0, n_paths)
  const double* guide_w;   // emission-guide weights [11433] or NULL (cosine emission)
  int32_t guide_bf16;      // 1: round MLP operands to bfloat16 where the GPU does
  int32_t guide_diffuse;   // 1 (with guide_w): Lambertian vertices scatter from the
                           // guide table of their texel (see build_guide_table)
  const uint8_t* guide_flag;  // test bookkeeping, or NULL: per guide-table entry, 1 marks
                              // it; ora_render's info bit 2 reports a path that scatters
                              // from a marked entry (changes nothing computed)
} ora_args;

}  // extern "C"

namespace {

const double kTmin = 1e-4, kEps = 1e-4, kInvPi = 0.31830988618379067154;
const double kLumR = 0.2126, kLumG = 0.7152, kLumB = 0.0722;

// ----------------------------------------------------------------- guide
// Learned emission guide (an extension; the paper samples emission
// cosine-weighted).  A multilayer perceptron 6 -> 64 -> 64 -> 64 -> 41 maps a
// light vertex (position normalised to the scene box, unit normal) to a
// mixture of 8 von Mises-Fisher lobes {mean m_k (3), log-concentration (1),
// logit (1)} and a mixing weight logit.  The sampling density is
//   q(w) = alpha * sum_k pi_k [v_k(w) + v_k(mirror(w))] + (1 - alpha) max(w.n, 0) / pi,
// the lobes folded onto the emitting hemisphere by the mirror about the
// emitter plane, with alpha = 0.9 sigmoid(o_40) so that the cosine part
// always keeps at least a tenth of the mass (bounded weights, positive
// density wherever emission is).  Parameter layout, row-major (out, in):
//   W1[64][6] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[41][64] b4[41].
// The GPU multiplies in bfloat16 with FP32 accumulation; with bf16 = true the
// oracle rounds exactly the operands the GPU rounds (weights, layer inputs,
// backward adjoints entering a product) and keeps everything else in FP64.
constexpr int kGIn = 6, kGH = 64, kGOut = 41, kGLobes = 8;
constexpr long kGW1 = 0, kGB1 = kGW1 + kGH * kGIn, kGW2 = kGB1 + kGH, kGB2 = kGW2 + kGH * kGH,
               kGW3 = kGB2 + kGH, kGB3 = kGW3 + kGH * kGH, kGW4 = kGB3 + kGH, kGB4 = kGW4 + kGOut * kGH,
               kGN = kGB4 + kGOut;
const double kLogKMin = -3.0, kLogKMax = 8.0, kAlphaMax = 0.9;

// Round to the nearest bfloat16 (8 significant bits), ties to even.
double bf16r(double x) {
  if (x == 0.0 || !std::isfinite(x)) return x;
  int e; std::frexp(x, &e);          // |x| in [2^(e-1), 2^e)
  double q = std::ldexp(1.0, e - 8);  // spacing of 8-bit significands there
  return std::nearbyint(x / q) * q;
}

struct GuideAct {
  double in[kGIn];
  double z1[kGH], h1[kGH], z2[kGH], h2[kGH], z3[kGH], h3[kGH];
  double o[kGOut];
};

// z[o] = sum_i W[o][i] x[i] + b[o], operands rounded when bf.
void glayer(const double* W, const double* b, const double* x, int n_in, int n_out, bool bf, double* z) {
  for (int o = 0; o < n_out; ++o) {
    double s = 0.0;
    for (int i = 0; i < n_in; ++i) s += (bf ? bf16r(W[o * n_in + i]) * bf16r(x[i]) : W[o * n_in + i] * x[i]);
    z[o] = s + b[o];
  }
}

void guide_forward(const double* w, const double feat[kGIn], bool bf, GuideAct& a) {
  for (int i = 0; i < kGIn; ++i) a.in[i] = feat[i];
  glayer(w + kGW1, w + kGB1, a.in, kGIn, kGH, bf, a.z1);
  for (int i = 0; i < kGH; ++i) a.h1[i] = std::max(a.z1[i], 0.0);
  glayer(w + kGW2, w + kGB2, a.h1, kGH, kGH, bf, a.z2);
  for (int i = 0; i < kGH; ++i) a.h2[i] = std::max(a.z2[i], 0.0);
  glayer(w + kGW3, w + kGB3, a.h2, kGH, kGH, bf, a.z3);
  for (int i = 0; i < kGH; ++i) a.h3[i] = std::max(a.z3[i], 0.0);
  glayer(w + kGW4, w + kGB4, a.h3, kGH, kGOut, bf, a.o);
}

// Scene box used to normalise guide positions: static triangles, the
// heightfield footprint at its base height and the emitter's corners.
void scene_box(const ora_scene* sc, double c[3], double h[3]) {
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  auto add = [&](double x, double y, double z) {
    double p[3] = {x, y, z};
    for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], p[k]); hi[k] = std::max(hi[k], p[k]); }
  };
  for (long i = 0; i < (long)sc->n_tris * 3; ++i) add(sc->tri_v[i * 3], sc->tri_v[i * 3 + 1], sc->tri_v[i * 3 + 2]);
  if (sc->hf_G > 1) {
    double ext = (sc->hf_G - 1) * sc->hf_dx;
    add(sc->hf_x0, sc->hf_base, sc->hf_z0);
    add(sc->hf_x0 + ext, sc->hf_base, sc->hf_z0 + ext);
  }
  const double* o = sc->em_o; const double* e1 = sc->em_e1; const double* e2 = sc->em_e2;
  add(o[0], o[1], o[2]);
  if (sc->em_type != ORA_EMIT_POINT) {
    add(o[0] + e1[0], o[1] + e1[1], o[2] + e1[2]);
    add(o[0] + e2[0], o[1] + e2[1], o[2] + e2[2]);
    add(o[0] + e1[0] + e2[0], o[1] + e1[1] + e2[1], o[2] + e1[2] + e2[2]);
  }
  for (int k = 0; k < 3; ++k) { c[k] = 0.5 * (lo[k] + hi[k]); h[k] = 0.5 * (hi[k] - lo[k]); }
}

void guide_features(const double c[3], const double h[3], D3 x, D3 n, double f[kGIn]) {
  double p[3] = {x.x, x.y, x.z};
  for (int k = 0; k < 3; ++k) f[k] = h[k] > 0.0 ? (p[k] - c[k]) / h[k] : 0.0;
  f[3] = n.x; f[4] = n.y; f[5] = n.z;
}

struct Mixture {
  D3 mu[kGLobes]; double mlen[kGLobes], kappa[kGLobes], pi[kGLobes];
  bool kfree[kGLobes];  // log-concentration inside its clamp range
  double alpha, sig;    // alpha = kAlphaMax * sig
};

Mixture mixture_of(const double o[kGOut]) {
  Mixture m;
  double lmax = -1e300;
  for (int k = 0; k < kGLobes; ++k) lmax = std::max(lmax, o[5 * k + 4]);
  double z = 0.0;
  for (int k = 0; k < kGLobes; ++k) {
    const double* q = o + 5 * k;
    double l = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    m.mlen[k] = l;
    m.mu[k] = l > 0.0 ? D3{q[0] / l, q[1] / l, q[2] / l} : D3{0.0, 0.0, 1.0};
    double lk = q[3];
    m.kfree[k] = lk > kLogKMin && lk < kLogKMax;
    m.kappa[k] = std::exp(std::min(std::max(lk, kLogKMin), kLogKMax));
    m.pi[k] = std::exp(q[4] - lmax);
    z += m.pi[k];
  }
  for (int k = 0; k < kGLobes; ++k) m.pi[k] /= z;
  m.sig = 1.0 / (1.0 + std::exp(-o[40]));
  m.alpha = kAlphaMax * m.sig;
  return m;
}

// von Mises-Fisher density on the unit sphere.
double vmf(D3 mu, double kappa, D3 w) {
  return kappa / (2.0 * M_PI * -std::expm1(-2.0 * kappa)) * std::exp(kappa * (dot(mu, w) - 1.0));
}

D3 mirror(D3 w, D3 n) { return w - n * (2.0 * dot(w, n)); }

double guide_pdf(const Mixture& m, D3 n, D3 w) {
  double c = dot(w, n);
  if (c < 0.0) return 0.0;
  D3 wm = mirror(w, n);
  double V = 0.0;
  for (int k = 0; k < kGLobes; ++k) V += m.pi[k] * (vmf(m.mu[k], m.kappa[k], w) + vmf(m.mu[k], m.kappa[k], wm));
  return m.alpha * V + (1.0 - m.alpha) * c * kInvPi;
}

// Draw a direction from the folded mixture with uniforms g0 (component),
// g1, g2 (direction).  comp: 0 cosine part, k + 1 lobe k.
// vMF sampling by inverting the cosine marginal (Wood 1994; Jakob 2012):
// t = 1 + log(xi + (1 - xi) e^{-2 kappa}) / kappa with xi = 1 - g1 in (0, 1].
D3 guide_sample(const Mixture& m, D3 n, double g0, double g1, double g2, int& comp) {
  if (g0 >= m.alpha) {
    comp = 0;
    double rr = std::sqrt(g1), phi = 2.0 * M_PI * g2;
    D3 t1, t2; onb(n, t1, t2);
    return t1 * (rr * std::cos(phi)) + t2 * (rr * std::sin(phi)) + n * std::sqrt(std::max(0.0, 1.0 - g1));
  }
  double v = g0 / m.alpha, acc = 0.0;
  int k = kGLobes - 1;
  for (int i = 0; i < kGLobes; ++i) { acc += m.pi[i]; if (v < acc) { k = i; break; } }
  comp = k + 1;
  double kap = m.kappa[k], xi = 1.0 - g1;
  double t = 1.0 + std::log(xi + (1.0 - xi) * std::exp(-2.0 * kap)) / kap;
  t = std::min(std::max(t, -1.0), 1.0);
  double s = std::sqrt(std::max(0.0, 1.0 - t * t)), phi = 2.0 * M_PI * g2;
  D3 t1, t2; onb(m.mu[k], t1, t2);
  D3 w = m.mu[k] * t + t1 * (s * std::cos(phi)) + t2 * (s * std::sin(phi));
  if (dot(w, n) < 0.0) w = mirror(w, n);
  return w;
}

// d(-c log q(w))/d o for one sample; returns -c log q (0 when q <= 0).
double guide_loss_grad_o(const double o[kGOut], D3 n, D3 w, double c, double g[kGOut]) {
  for (int i = 0; i < kGOut; ++i) g[i] = 0.0;
  if (c == 0.0) return 0.0;
  Mixture m = mixture_of(o);
  double q = guide_pdf(m, n, w);
  if (!(q > 0.0)) return 0.0;
  double cosp = std::max(dot(w, n), 0.0) * kInvPi;
  D3 wm = mirror(w, n);
  D3 ws[2] = {w, wm};
  double Vk[kGLobes], V = 0.0;
  for (int k = 0; k < kGLobes; ++k) {
    Vk[k] = vmf(m.mu[k], m.kappa[k], w) + vmf(m.mu[k], m.kappa[k], wm);
    V += m.pi[k] * Vk[k];
  }
  double s = -c / q;  // d(-c log q)/dq
  // alpha = kAlphaMax * sigmoid(o_40)
  g[40] = s * (V - cosp) * kAlphaMax * m.sig * (1.0 - m.sig);
  for (int k = 0; k < kGLobes; ++k) {
    double wk = s * m.alpha * m.pi[k];
    g[5 * k + 4] = s * m.alpha * m.pi[k] * (Vk[k] - V);  // softmax logits
    double kap = m.kappa[k], dk = 0.0;
    double gm[3] = {0.0, 0.0, 0.0};
    for (int r = 0; r < 2; ++r) {
      double mw = dot(m.mu[k], ws[r]);
      double v = vmf(m.mu[k], kap, ws[r]);
      dk += v * (1.0 / kap - 2.0 / std::expm1(2.0 * kap) + (mw - 1.0));
      if (m.mlen[k] > 0.0) {
        D3 t = (ws[r] - m.mu[k] * mw) * (v * kap / m.mlen[k]);
        gm[0] += t.x; gm[1] += t.y; gm[2] += t.z;
      }
    }
    g[5 * k + 3] = m.kfree[k] ? wk * dk * kap : 0.0;
    for (int a = 0; a < 3; ++a) g[5 * k + a] = wk * gm[a];
  }
  return -c * std::log(q);
}

// Accumulate the parameter gradient of one sample given d(loss)/d(outputs).
void guide_backward(const double* w, const GuideAct& a, const double go[kGOut], bool bf, double* grad) {
  auto r = [bf](double x) { return bf ? bf16r(x) : x; };
  double dz4[kGOut], dz3[kGH], dz2[kGH], dz1[kGH];
  for (int o = 0; o < kGOut; ++o) dz4[o] = go[o];
  auto back = [&](const double* W, int n_in, int n_out, const double* dz, const double* xin, long oW, long oB,
                  const double* zprev, double* dzprev) {
    for (int o = 0; o < n_out; ++o) {
      grad[oB + o] += dz[o];
      for (int i = 0; i < n_in; ++i) grad[oW + (long)o * n_in + i] += r(dz[o]) * r(xin[i]);
    }
    if (!dzprev) return;
    for (int i = 0; i < n_in; ++i) {
      double s = 0.0;
      for (int o = 0; o < n_out; ++o) s += r(W[(long)o * n_in + i]) * r(dz[o]);
      dzprev[i] = zprev[i] > 0.0 ? s : 0.0;
    }
  };
  back(w + kGW4, kGH, kGOut, dz4, a.h3, kGW4, kGB4, a.z3, dz3);
  back(w + kGW3, kGH, kGH, dz3, a.h2, kGW3, kGB3, a.z2, dz2);
  back(w + kGW2, kGH, kGH, dz2, a.h1, kGW2, kGB2, a.z1, dz1);
  back(w + kGW1, kGIn, kGH, dz1, a.in, kGW1, kGB1, nullptr, nullptr);
}

struct Scene {
  const ora_scene* s;
  int n_static, n_hf, n_all;
  const double* albedo; const double* Le; const double* heights;
  const double* nmap;   // [G][G][2] normal-map slopes (Sx, Sz), or null: slopes from the heights
  bool attached;
  long slot_Le, slot_h, slot_n;
  long n_le;            // emitter radiance parameters: 3, or 3 per texel of a textured emitter
  std::vector<D3> tv;   // [n_all][3] primal vertex positions
  // camera frame
  D3 cpos, f, r, u; double tan_half, aspect, K_area;
  double gc[3], gh[3];  // guide position normalisation (scene box centre, half extent)
  // guide table of the Lambertian texels (built by build_guide_table)
  std::vector<Mixture> gtab;
  std::vector<uint8_t> gok;

  int hf_corner(int tri, int k, int& gi, int& gj) const {
    // heightfield triangle -> grid corner (gi, gj); returns 1 if on heightfield
    int local = tri - n_static;
    int cell = local >> 1, half = local & 1, G = s->hf_G;
    int ci = cell % (G - 1), cj = cell / (G - 1);
    // half 0: (A, C, B); half 1: (A, D, C) with A=(i,j) B=(i+1,j) C=(i+1,j+1) D=(i,j+1)
    static const int o0[3][2] = {{0, 0}, {1, 1}, {1, 0}};
    static const int o1[3][2] = {{0, 0}, {0, 1}, {1, 1}};
    const int (*o)[2] = half == 0 ? o0 : o1;
    gi = ci + o[k][0]; gj = cj + o[k][1];
    return 1;
  }
  double hval(int gi, int gj) const { return heights ? heights[gj * s->hf_G + gi] : 0.0; }
  V hvar(int gi, int gj) const {
    double v = hval(gi, gj);
    if (attached) return leaf(v, slot_h + (long)gj * s->hf_G + gi);
    return V(v);
  }

  void init(const ora_scene* sc, const double* alb, const double* le, const double* h, const double* nm, bool att) {
    s = sc; albedo = alb; Le = le; heights = h; attached = att && sc->hf_G > 1 && h;
    nmap = sc->hf_G > 1 ? nm : nullptr;
    n_static = sc->n_tris;
    n_hf = sc->hf_G > 1 ? 2 * (sc->hf_G - 1) * (sc->hf_G - 1) : 0;
    n_all = n_static + n_hf;
    slot_Le = (long)sc->n_tex * sc->tex_res * sc->tex_res * 3;
    n_le = 3L * (sc->em_tex_res > 0 ? (long)sc->em_tex_res * sc->em_tex_res : 1);
    slot_h = slot_Le + n_le;
    slot_n = slot_h + (sc->hf_G > 1 ? (long)sc->hf_G * sc->hf_G : 0);
    tv.resize((size_t)n_all * 3);
    for (int t = 0; t < n_static; ++t)
      for (int k = 0; k < 3; ++k)
        tv[t * 3 + k] = {sc->tri_v[(t * 3 + k) * 3 + 0], sc->tri_v[(t * 3 + k) * 3 + 1],
                         sc->tri_v[(t * 3 + k) * 3 + 2]};
    for (int t = n_static; t < n_all; ++t)
      for (int k = 0; k < 3; ++k) {
        int gi, gj; hf_corner(t, k, gi, gj);
        tv[t * 3 + k] = {sc->hf_x0 + gi * sc->hf_dx, sc->hf_base + hval(gi, gj),
                         sc->hf_z0 + gj * sc->hf_dx};
      }
    cpos = {sc->cam_pos[0], sc->cam_pos[1], sc->cam_pos[2]};
    D3 tgt = {sc->cam_target[0], sc->cam_target[1], sc->cam_target[2]};
    D3 up = {sc->cam_up[0], sc->cam_up[1], sc->cam_up[2]};
    f = normalize(tgt - cpos);
    r = normalize(cross(f, up));
    u = cross(r, f);
    tan_half = std::tan(sc->cam_fov_deg * M_PI / 360.0);
    aspect = (double)sc->width / (double)sc->height;
    scene_box(sc, gc, gh);
  }

  int mat_of(int tri) const { return tri < n_static ? s->tri_mat[tri] : s->hf_mat; }

  // Closest hit (discrete choice), brute force over every triangle.
  // Moller-Trumbore with inclusive edges; ties go to the lower index.
  int closest(D3 o, D3 d, double tmin, double tmax, double* t_out) const {
    int best = -1; double bt = tmax;
    for (int t = 0; t < n_all; ++t) {
      D3 p0 = tv[t * 3], e1 = tv[t * 3 + 1] - p0, e2 = tv[t * 3 + 2] - p0;
      D3 pv = cross(d, e2);
      double det = dot(e1, pv);
      if (std::fabs(det) < 1e-300) continue;
      double inv = 1.0 / det;
      D3 tvec = o - p0;
      double b1 = dot(tvec, pv) * inv;
      if (b1 < 0.0 || b1 > 1.0) continue;
      D3 q = cross(tvec, e1);
      double b2 = dot(d, q) * inv;
      if (b2 < 0.0 || b1 + b2 > 1.0) continue;
      double tt = dot(e2, q) * inv;
      if (tt > tmin && tt < bt) { bt = tt; best = t; }
    }
    if (t_out) *t_out = bt;
    return best;
  }

  // Differentiable triangle corners.
  void corners(int tri, V3 P[3]) const {
    if (tri < n_static) {
      for (int k = 0; k < 3; ++k) P[k] = cst(tv[tri * 3 + k]);
      return;
    }
    for (int k = 0; k < 3; ++k) {
      int gi, gj; hf_corner(tri, k, gi, gj);
      P[k] = {V(s->hf_x0 + gi * s->hf_dx), V(s->hf_base) + hvar(gi, gj), V(s->hf_z0 + gj * s->hf_dx)};
    }
  }

  // Shading slopes at grid vertex (gi, gj): the normal-map parameters when
  // the surface is normal-mapped, else the central-difference slope of the
  // heightfield, one-sided on the border.
  void slope(int gi, int gj, V& sx, V& sz) const {
    int G = s->hf_G; double dx = s->hf_dx;
    if (nmap) {
      long k = 2 * ((long)gj * G + gi);
      sx = attached ? leaf(nmap[k], slot_n + k) : V(nmap[k]);
      sz = attached ? leaf(nmap[k + 1], slot_n + k + 1) : V(nmap[k + 1]);
      return;
    }
    int a = std::max(gi - 1, 0), b = std::min(gi + 1, G - 1);
    sx = (hvar(b, gj) - hvar(a, gj)) / V((b - a) * dx);
    int c = std::max(gj - 1, 0), d = std::min(gj + 1, G - 1);
    sz = (hvar(gi, d) - hvar(gi, c)) / V((d - c) * dx);
  }
};

// Centre of every albedo texel on the scene surface, for the diffuse guide
// table.  Texel (t, tx, ty) has chart centre ((tx + 1/2)/R, (ty + 1/2)/R);
// its position and unit normal come from the lowest-index static triangle
// whose material is Lambertian with texture t and whose chart triangle
// contains the centre (barycentrics >= -1e-9): the barycentric blend of its
// corners and normalize((v1 - v0) x (v2 - v0)).  ok[texel] = 0 when no
// triangle covers the centre.  x, n: [n_tex R R][3].
void texel_centres(const ora_scene* sc, std::vector<double>& x, std::vector<double>& n, std::vector<uint8_t>& ok) {
  const int R = sc->tex_res;
  const long T = (long)sc->n_tex * R * R;
  x.assign(T * 3, 0.0); n.assign(T * 3, 0.0); ok.assign(T, 0);
  for (int t = 0; t < sc->n_tris; ++t) {
    int mat = sc->tri_mat[t];
    if (sc->mat_type[mat] != ORA_LAMBERT) continue;
    int tex = sc->mat_tex[mat];
    const double* uv = sc->tri_uv + (size_t)t * 6;
    const double* v = sc->tri_v + (size_t)t * 9;
    double a0 = uv[2] - uv[0], a1 = uv[3] - uv[1], b0 = uv[4] - uv[0], b1 = uv[5] - uv[1];
    double det = a0 * b1 - a1 * b0;
    if (std::fabs(det) < 1e-300) continue;
    D3 p0 = {v[0], v[1], v[2]}, p1 = {v[3], v[4], v[5]}, p2 = {v[6], v[7], v[8]};
    D3 nrm = normalize(cross(p1 - p0, p2 - p0));
    for (int ty = 0; ty < R; ++ty)
      for (int tx = 0; tx < R; ++tx) {
        long k = ((long)tex * R + ty) * R + tx;
        if (ok[k]) continue;
        double cx = (tx + 0.5) / R - uv[0], cy = (ty + 0.5) / R - uv[1];
        double l1 = (cx * b1 - cy * b0) / det, l2 = (a0 * cy - a1 * cx) / det, l0 = 1.0 - l1 - l2;
        if (l0 < -1e-9 || l1 < -1e-9 || l2 < -1e-9) continue;
        D3 c = p0 * l0 + p1 * l1 + p2 * l2;
        x[k * 3] = c.x; x[k * 3 + 1] = c.y; x[k * 3 + 2] = c.z;
        n[k * 3] = nrm.x; n[k * 3 + 1] = nrm.y; n[k * 3 + 2] = nrm.z;
        ok[k] = 1;
      }
  }
}

// Guide table (an extension, like the emission guide): the mixture of the
// network at each texel centre, entry 2 texel + side with the network's
// normal input +n (side 0) or -n (side 1).  A Lambertian vertex that the
// ray reaches against its triangle's geometric normal (cos_in < 0) uses
// side 0, else side 1; a vertex of an uncovered texel samples the cosine
// density.  Raw outputs of every entry go to `raw` when given.
void build_guide_table(Scene& S, const ora_args& A, std::vector<double>* raw) {
  std::vector<double> x, n; std::vector<uint8_t> ok;
  texel_centres(S.s, x, n, ok);
  const long T = (long)ok.size();
  S.gtab.assign(2 * T, Mixture{});
  S.gok.assign(2 * T, 0);
  if (raw) raw->assign(2 * T * kGOut, 0.0);
  for (long k = 0; k < T; ++k) {
    if (!ok[k]) continue;
    for (int side = 0; side < 2; ++side) {
      double sg = side ? -1.0 : 1.0;
      D3 xc = {x[k * 3], x[k * 3 + 1], x[k * 3 + 2]}, nc = {sg * n[k * 3], sg * n[k * 3 + 1], sg * n[k * 3 + 2]};
      double f[kGIn]; guide_features(S.gc, S.gh, xc, nc, f);
      GuideAct act; guide_forward(A.guide_w, f, A.guide_bf16 != 0, act);
      S.gtab[2 * k + side] = mixture_of(act.o);
      S.gok[2 * k + side] = 1;
      if (raw) for (int q = 0; q < kGOut; ++q) (*raw)[(2 * k + side) * kGOut + q] = act.o[q];
    }
  }
}

// Scattering at a smooth dielectric interface (the Glass Slab / caustic
// material of Sec. 6), as an AD expression of the incoming direction w_in and
// the unit shading normal ns (same side as the unit geometric normal ng).
// The lobe is chosen with the unpolarized Fresnel reflectance F (textbook
// s/p amplitudes, relative index eta = n_from / n_to): reflect iff
// u_lobe < F, else refract by Snell's law; either lobe has weight 1, so the
// throughput is unchanged.  Returns 7 (and no direction) when w_in arrives
// from behind the shading normal, 8 when the new direction falls on the wrong
// side of the geometric normal (the path ends), else 0.
int dielectric_event(const V3& w_in, const V3& ns, D3 ng, double ior, double u_lobe, V3& wo, bool& reflect,
                     double& F) {
  const double cos_g = dot(val(w_in), ng);
  const bool entering = cos_g < 0.0;
  const double eta = entering ? 1.0 / ior : ior;
  const V3 n = entering ? ns : ns * V(-1.0);
  const V cosi = -dot(w_in, n);
  reflect = false;
  F = 0.0;
  if (cosi.v <= 0.0) return 7;
  const double sin2t = eta * eta * (1.0 - cosi.v * cosi.v);
  if (sin2t >= 1.0) {
    F = 1.0;  // total internal reflection
  } else {
    const double cost_d = std::sqrt(1.0 - sin2t);
    const double ei = entering ? 1.0 : ior, et = entering ? ior : 1.0;
    const double rs = (ei * cosi.v - et * cost_d) / (ei * cosi.v + et * cost_d);
    const double rp = (et * cosi.v - ei * cost_d) / (et * cosi.v + ei * cost_d);
    F = 0.5 * (rs * rs + rp * rp);
  }
  reflect = u_lobe < F;
  if (reflect) {
    wo = w_in + n * (V(2.0) * cosi);
  } else {
    const V cost = vsqrt(V(1.0) - V(eta * eta) * (V(1.0) - cosi * cosi));
    wo = w_in * V(eta) + n * (V(eta) * cosi - cost);
  }
  const double side_in = -cos_g;  // > 0 when the ray arrived on the +ng side
  const double s_out = dot(val(wo), ng);
  if (reflect ? (s_out * side_in <= 0.0) : (s_out * side_in >= 0.0)) return 8;
  return 0;
}

// Rough conductor (an extension for the Mirror validation of Sec. 6.1: the
// paper names a roughened conductor without fixing its model).  GGX /
// Trowbridge-Reitz microfacets of roughness a about the unit shading normal
// n, Smith's separable masking, and a reflectance F0 (the material's albedo
// texel) that does not vary with angle:
//   D(m) = a^2 / (pi ((m.n)^2 (a^2 - 1) + 1)^2),
//   G1(v) = 2 (v.n) / ((v.n) + sqrt(a^2 + (1 - a^2)(v.n)^2)),
//   f(wi, wo) = F0 D(h) G1(wi) G1(wo) / (4 (wi.n)(wo.n)),  h = normalize(wi + wo).
// Sampling draws m with density D(m)(m.n) (tan^2 theta_m = a^2 u0 / (1 - u0),
// phi = 2 pi u1) and reflects wi about it; the weight f (wo.n) / p is then
// F0 G1(wi) G1(wo) (wi.m) / ((wi.n)(m.n)).
V ggx_D(const V& cm, double a2) {
  V d = cm * cm * V(a2 - 1.0) + V(1.0);
  return V(a2 * kInvPi) / (d * d);
}
V ggx_G1(const V& cv, double a2) { return V(2.0) * cv / (cv + vsqrt(V(a2) + V(1.0 - a2) * cv * cv)); }

// local microfacet normal (x, y, z) of the uniforms (u0, u1)
void ggx_local(double a, double u0, double u1, double& lx, double& ly, double& lz) {
  double t2 = a * a * u0 / (1.0 - u0);
  lz = 1.0 / std::sqrt(1.0 + t2);
  double st = std::sqrt(std::max(0.0, 1.0 - lz * lz)), phi = 2.0 * M_PI * u1;
  lx = st * std::cos(phi); ly = st * std::sin(phi);
}

// The conductor's part of a sensor connection from the vertex, f (wc.n) / F0
// = D(h) G1(wi) G1(wc) / (4 wi.n), for unit wi, wc on the side of n.
V conductor_conn(const V3& wi, const V3& wc, const V3& n, double a) {
  const double a2 = a * a;
  V3 h = normalize(wi + wc);
  V cosi = dot(wi, n);
  return ggx_D(dot(h, n), a2) * ggx_G1(cosi, a2) * ggx_G1(dot(wc, n), a2) / (V(4.0) * cosi);
}

// Microfacet reflection of unit wi (pointing away from the surface, on the
// side of the unit shading normal n) with the microfacet normal of (u0, u1)
// held fixed in the local frame of n: writes wo and the weight f (wo.n) / p
// over F0.  Returns 7 when wi does not see the drawn microfacet, 8 when wo
// leaves below n or on the far side of the geometric normal ng (side_in =
// +1 when the ray arrived on the +ng side), else 0.
int conductor_event(const V3& wi, const V3& n, D3 ng, double side_in, double a, double u0, double u1, V3& wo,
                    V& wgt) {
  const double a2 = a * a;
  double lx, ly, lz;
  ggx_local(a, u0, u1, lx, ly, lz);
  V3 t1, t2; onbv(n, t1, t2);
  V3 m = t1 * V(lx) + t2 * V(ly) + n * V(lz);
  V cwm = dot(wi, m);
  if (cwm.v <= 0.0) return 7;
  wo = m * (V(2.0) * cwm) - wi;
  V coso = dot(wo, n);
  if (coso.v <= 0.0 || dot(val(wo), ng) * side_in <= 0.0) return 8;
  V cosi = dot(wi, n);
  wgt = ggx_G1(cosi, a2) * ggx_G1(coso, a2) * cwm / (cosi * V(lz));
  return 0;
}

struct Conn { V C[3]; V ux, uy; int depth; };

struct PathResult {
  std::vector<Conn> conns;
  uint32_t sig; int R; double W;
  // An ill-conditioned vertex lies at or before the path's last sensor
  // connection: a grazing hit (|cos| < 0.02), a segment shorter than 0.02
  // scene units, a refraction with cos_t < 0.1, or a connection within
  // 1e-3 px of a kink of the tent filter.  Test bookkeeping only (the
  // derivatives of such paths amplify rounding by 1/cos^2, 1/length or a
  // one-sided filter slope); it changes nothing the oracle computes.
  bool illc;
  // first guided Lambertian scatter of the path (guide training sample):
  // vertex depth (0: none), position, arrival-side normal, direction,
  // density, component
  int gdepth; double gx[3], gn[3], gwd[3], gq; int gcomp;
  bool gflag;  // scattered from a guide-table entry marked in ora_args.guide_flag
};

inline bool near_tent_kink(double u) {
  double d = u - 0.5;
  return std::fabs(d - std::nearbyint(d)) < 1e-3;
}

// Trace one light path as an AD expression of the parameters.
void trace_path(const Scene& S, const ora_args& A, uint32_t path, PathResult& out) {
  const ora_scene& sc = *S.s;
  out.conns.clear(); out.sig = 0x811C9DC5u; out.R = 0; out.W = 0.0; out.illc = false; out.gdepth = 0; out.gflag = false;
  bool ill = false;  // ill-conditioned vertex so far
  const int W = sc.width, H = sc.height;
  const double Kfilm = (double)W * H / (4.0 * S.aspect * S.tan_half * S.tan_half * (double)A.n_paths);

  // --- emission (vertex 0)
  Uniform4 u0 = rng4(A.seed, path, 0, 0);
  // radiance of the emission point: the texel of its quad coordinates (u0
  // along e1, u1 along e2; nearest texel) when the emitter is textured
  long le = 0;
  if (sc.em_tex_res > 0) {
    const int R = sc.em_tex_res;
    int tx = std::min((int)std::floor(u0.u[0] * R), R - 1), ty = std::min((int)std::floor(u0.u[1] * R), R - 1);
    le = 3L * ((long)ty * R + tx);
  }
  V Le[3];
  for (int c = 0; c < 3; ++c) Le[c] = leaf(S.Le[le + c], S.slot_Le + le + c);
  D3 x0, w0, n_off; bool has_off;
  V beta[3];
  if (sc.em_type == ORA_EMIT_DIRECTIONAL) {
    // a collimated beam leaving the quad along its normal: irradiance Le
    // across the quad, uniform position, beta_1 = Le * area
    D3 o = {sc.em_o[0], sc.em_o[1], sc.em_o[2]};
    D3 e1 = {sc.em_e1[0], sc.em_e1[1], sc.em_e1[2]}, e2 = {sc.em_e2[0], sc.em_e2[1], sc.em_e2[2]};
    D3 cr = cross(e1, e2);
    double area = std::sqrt(dot(cr, cr));
    D3 ne = cr * (1.0 / area);
    x0 = o + e1 * u0.u[0] + e2 * u0.u[1];
    w0 = ne;
    n_off = ne; has_off = true;
    for (int c = 0; c < 3; ++c) beta[c] = Le[c] * V(area);
  } else if (sc.em_type == ORA_EMIT_QUAD) {
    D3 o = {sc.em_o[0], sc.em_o[1], sc.em_o[2]};
    D3 e1 = {sc.em_e1[0], sc.em_e1[1], sc.em_e1[2]}, e2 = {sc.em_e2[0], sc.em_e2[1], sc.em_e2[2]};
    D3 cr = cross(e1, e2);
    double area = std::sqrt(dot(cr, cr));
    D3 ne = cr * (1.0 / area);
    x0 = o + e1 * u0.u[0] + e2 * u0.u[1];
    double rr = std::sqrt(u0.u[2]), phi = 2.0 * M_PI * u0.u[3];
    double lx = rr * std::cos(phi), ly = rr * std::sin(phi), lz = std::sqrt(std::max(0.0, 1.0 - u0.u[2]));
    D3 t1, t2; onb(ne, t1, t2);
    w0 = t1 * lx + t2 * ly + ne * lz;
    n_off = ne; has_off = true;
    double fac = area * M_PI;
    if (A.guide_w) {  // guided emission: direction from the mixture, weight cos / q
      double feat[kGIn]; guide_features(S.gc, S.gh, x0, ne, feat);
      GuideAct act; guide_forward(A.guide_w, feat, A.guide_bf16 != 0, act);
      Mixture m = mixture_of(act.o);
      Uniform4 g = rng4(A.seed, path, 0, 1);
      int comp;
      w0 = guide_sample(m, ne, g.u[0], g.u[1], g.u[2], comp);
      double q = guide_pdf(m, ne, w0);
      fac = q > 0.0 ? area * dot(w0, ne) / q : 0.0;
    }
    for (int c = 0; c < 3; ++c) beta[c] = Le[c] * V(fac);
  } else {
    x0 = {sc.em_o[0], sc.em_o[1], sc.em_o[2]};
    double z = 1.0 - 2.0 * u0.u[2];
    double rr = std::sqrt(std::max(0.0, 1.0 - z * z)), phi = 2.0 * M_PI * u0.u[3];
    w0 = {rr * std::cos(phi), rr * std::sin(phi), z};
    n_off = {0, 0, 0}; has_off = false;
    for (int c = 0; c < 3; ++c) beta[c] = Le[c] * V(4.0 * M_PI);
  }

  V3 xprev = cst(x0), wcur = cst(w0);
  D3 offn = n_off; bool off = has_off;
  double Omega = 0.0, omegaR = 0.0;

  for (int j = 1; j <= A.max_depth; ++j) {
    // --- closest hit (discrete) from the offset origin
    D3 xo = val(xprev), wd = val(wcur);
    if (off) xo = xo + offn * (dot(wd, offn) >= 0 ? kEps : -kEps);
    double th;
    int tri = S.closest(xo, wd, kTmin, 1e300, &th);
    if (tri < 0) { out.sig = fnv1a(out.sig, 0u); break; }
    out.sig = fnv1a(out.sig, (uint32_t)tri + 1u);
    int mat = S.mat_of(tri);
    int mtype = sc.mat_type[mat];
    if (mtype == ORA_ABSORBER) break;

    // --- differentiable hit point from the true origin
    V3 P[3]; S.corners(tri, P);
    V3 e1 = P[1] - P[0], e2 = P[2] - P[0];
    V3 N = cross(e1, e2);
    V t = dot(P[0] - xprev, N) / dot(wcur, N);
    V3 x = xprev + wcur * t;
    V nn = dot(N, N);
    V3 dx = x - P[0];
    V b1 = dot(cross(dx, e2), N) / nn;
    V b2 = dot(cross(e1, dx), N) / nn;
    V3 ng = normalize(N);
    D3 ngd = val(ng), wd_in = val(wcur);
    double cos_in = dot(wd_in, ngd);
    Uniform4 uj = rng4(A.seed, path, (uint32_t)j, 0);
    {
      D3 seg = val(x) - val(xprev);
      if (std::fabs(cos_in) < 0.02 || dot(seg, seg) < 4e-4) ill = true;
    }

    // shading normal: the geometric one, or on the heightfield the
    // normalised (-S_x, 1, -S_z) of the barycentric blend of the vertex
    // slopes (central differences of the heights, or a normal map)
    auto shading_normal = [&]() {
      V3 ns = ng;
      if (tri >= S.n_static) {
        V sx[3], sz[3];
        for (int k = 0; k < 3; ++k) { int gi, gj; S.hf_corner(tri, k, gi, gj); S.slope(gi, gj, sx[k], sz[k]); }
        V c0 = V(1.0) - b1 - b2;
        V Sx = c0 * sx[0] + b1 * sx[1] + b2 * sx[2];
        V Sz = c0 * sz[0] + b1 * sz[1] + b2 * sz[2];
        ns = normalize(V3{-Sx, V(1.0), -Sz});
      }
      return ns;
    };

    if (mtype == ORA_LAMBERT || mtype == ORA_CONDUCTOR) {
      const bool cond = mtype == ORA_CONDUCTOR;
      // texel (nearest), from primal chart coordinates
      int tex = sc.mat_tex[mat], R = sc.tex_res;
      double uvx, uvy;
      if (tri < S.n_static) {
        const double* uv = sc.tri_uv + (size_t)tri * 6;
        double c0 = 1.0 - b1.v - b2.v;
        uvx = c0 * uv[0] + b1.v * uv[2] + b2.v * uv[4];
        uvy = c0 * uv[1] + b1.v * uv[3] + b2.v * uv[5];
      } else { uvx = uvy = 0.0; }
      int tx = (int)std::floor(uvx * R), ty = (int)std::floor(uvy * R);
      tx = std::min(std::max(tx, 0), R - 1); ty = std::min(std::max(ty, 0), R - 1);
      long texel = ((long)tex * R + ty) * R + tx;
      out.sig = fnv1a(out.sig, (uint32_t)texel + 1u);
      V rho[3];
      for (int c = 0; c < 3; ++c) rho[c] = leaf(S.albedo[texel * 3 + c], texel * 3 + c);
      // conductor: arrival-side shading normal n_a and wi = -w; a ray
      // arriving from behind n_a ends the path (no connection; code 9)
      V3 n_a = ng, wi = wcur * V(-1.0);
      V cosi(0.0);
      const double a_r = cond ? sc.mat_ior[mat] : 0.0;
      if (cond) {
        V3 ns = shading_normal();
        n_a = cos_in < 0 ? ns : ns * V(-1.0);
        cosi = dot(wi, n_a);
        if (cosi.v <= 0.0) { out.sig = fnv1a(out.sig, 9u); break; }
      }

      // --- sensor connection (Eq. 1 term i)
      uint32_t valid = 0;
      V3 dv = x - cst(S.cpos);
      V zc = dot(dv, cst(S.f));
      if (zc.v > 0.0) {
        V qx = dot(dv, cst(S.r)) / zc, qy = dot(dv, cst(S.u)) / zc;
        V ux = V(0.5 * W) * (V(1.0) + qx / V(S.aspect * S.tan_half));
        V uy = V(0.5 * H) * (V(1.0) - qy / V(S.tan_half));
        if (ux.v >= 0.0 && ux.v < W && uy.v >= 0.0 && uy.v < H) {
          D3 dvd = val(dv);
          double dist = std::sqrt(dot(dvd, dvd));
          D3 wc = dvd * (-1.0 / dist);
          double cg = dot(ngd, wc);
          const bool side_ok = cg * (-cos_in) > 0.0 && (!cond || dot(val(n_a), wc) > 0.0);
          if (side_ok) {
            D3 so = val(x) + ngd * (cg >= 0 ? kEps : -kEps);
            D3 sd = S.cpos - so;
            double sl = std::sqrt(dot(sd, sd));
            sd = sd * (1.0 / sl);
            if (S.closest(so, sd, kTmin, sl * (1.0 - 1e-4), nullptr) < 0) {
              valid = 1;
              V dist2 = dot(dv, dv);
              V distv = vsqrt(dist2);
              V cosc = zc / distv;
              V g;
              if (!cond) {
                V cosx = vabs(dot(ng, dv)) / distv;
                g = V(kInvPi * Kfilm) * cosx / (cosc * cosc * cosc * dist2);
              } else {
                V bc = conductor_conn(wi, dv * (V(-1.0) / distv), n_a, a_r);
                g = V(Kfilm) * bc / (cosc * cosc * cosc * dist2);
              }
              Conn cn;
              for (int c = 0; c < 3; ++c) cn.C[c] = beta[c] * rho[c] * g;
              cn.ux = ux; cn.uy = uy; cn.depth = j;
              // reservoir (Eq. 8): luminance weight, replace w.p. omega/Omega
              double om = kLumR * cn.C[0].v + kLumG * cn.C[1].v + kLumB * cn.C[2].v;
              if (om > 0.0) {
                Omega += om;
                if (uj.u[3] < om / Omega) { out.R = j; omegaR = om; }
              }
              out.conns.push_back(cn);
              if (near_tent_kink(ux.v) || near_tent_kink(uy.v)) ill = true;
              out.illc = ill;
            }
          }
        }
      }
      out.sig = fnv1a(out.sig, valid);
      if (j == A.max_depth) break;

      if (cond) {
        // --- microfacet reflection (the microfacet normal held fixed in the
        // local frame of n_a, so the frame moves with the surface)
        V3 wo; V wgt;
        int code = conductor_event(wi, n_a, ngd, cos_in < 0 ? 1.0 : -1.0, a_r, uj.u[0], uj.u[1], wo, wgt);
        if (code) { out.sig = fnv1a(out.sig, (uint32_t)code); break; }
        for (int c = 0; c < 3; ++c) beta[c] = beta[c] * rho[c] * wgt;
        xprev = x; wcur = wo;
        offn = ngd; off = true;
        continue;
      }
      // --- cosine-weighted scatter on the arrival side
      double rr = std::sqrt(uj.u[0]), phi = 2.0 * M_PI * uj.u[1];
      double lx = rr * std::cos(phi), ly = rr * std::sin(phi), lz = std::sqrt(std::max(0.0, 1.0 - uj.u[0]));
      V3 nav = cos_in < 0 ? ng : ng * V(-1.0);
      double gwf = 1.0;  // f cos / p over rho: 1 for cosine sampling
      const long ge = 2 * texel + (cos_in < 0 ? 0 : 1);
      if (A.guide_w && A.guide_diffuse && S.gok[ge]) {
        // guided scatter: direction from the texel's mixture folded about
        // the arrival-side normal (component by u2, direction by u0, u1),
        // weight cos / (pi q) with the density held fixed; the direction
        // enters the derivatives through its local coordinates, like the
        // cosine sample
        D3 nd = val(nav);
        if (A.guide_flag && A.guide_flag[ge]) out.gflag = true;
        int comp;
        D3 w = guide_sample(S.gtab[ge], nd, uj.u[2], uj.u[0], uj.u[1], comp);
        double q = guide_pdf(S.gtab[ge], nd, w), c = dot(w, nd);
        if (!(q > 0.0 && c > 0.0)) break;
        gwf = c / (M_PI * q);
        D3 b1p, b2p; onb(nd, b1p, b2p);
        lx = dot(w, b1p); ly = dot(w, b2p); lz = c;
        if (out.gdepth == 0) {
          D3 xp = val(x);
          out.gdepth = j;
          out.gx[0] = xp.x; out.gx[1] = xp.y; out.gx[2] = xp.z;
          out.gn[0] = nd.x; out.gn[1] = nd.y; out.gn[2] = nd.z;
          out.gwd[0] = w.x; out.gwd[1] = w.y; out.gwd[2] = w.z;
          out.gq = q; out.gcomp = comp;
        }
      }
      // the sampled direction is held fixed in the local frame of the
      // arrival-side normal, so the frame moves with the surface
      V3 t1, t2; onbv(nav, t1, t2);
      V3 wo = t1 * V(lx) + t2 * V(ly) + nav * V(lz);
      for (int c = 0; c < 3; ++c) beta[c] = beta[c] * rho[c] * V(gwf);
      xprev = x; wcur = wo;
      offn = ngd; off = true;
    } else {  // dielectric: Fresnel-sampled reflect / refract, weight 1
      V3 ns = shading_normal();
      if (j == A.max_depth) break;
      V3 wo;
      bool reflect = false;
      double F = 0.0;
      int code = dielectric_event(wcur, ns, ngd, sc.mat_ior[mat], uj.u[2], wo, reflect, F);
      if (code == 7) { out.sig = fnv1a(out.sig, 7u); break; }
      if (!reflect && std::fabs(dot(val(wo), val(ns))) < 0.1) ill = true;  // refraction near the critical angle
      out.sig = fnv1a(out.sig, reflect ? 2u : 4u);
      if (code == 8) { out.sig = fnv1a(out.sig, 8u); break; }
      xprev = x; wcur = wo;
      offn = ngd; off = true;
    }
  }
  if (out.R > 0) out.W = Omega / omegaR;
  out.sig = fnv1a(out.sig, (uint32_t)out.R);
}

// ----------------------------------------------------------------- camera side
// Camera paths for the bidirectional combination (an extension: the paper
// names PRB on the camera side with LRB-3-pass on the light side as its next
// step, without fixing an algorithm).  The light tracer connects only its
// non-specular vertices to the camera, so it misses exactly the paths whose
// first camera-side vertex is specular (seen through or in glass).  A camera
// path tracer restricted to those paths (spec_only) adds them; the two sets
// are disjoint and together hold every path the camera can see (emitters
// seen directly stay out of both, as in the light tracer).
//   Camera sample s: pixel p = s mod (W H), film position u = p + 1/2 + t
//   with t drawn from the tent filter (so E[estimate] = int F(u, p) L(u) du,
//   the light tracer's pixel), one radiance estimate per sample, each pixel
//   averaging spp = n_paths / (W H) samples.
//   Vertex j: dielectric -> Fresnel lobe (weight 1); Lambertian or rough
//   conductor -> next-event estimation to the emitter (a uniform point on a
//   quad emitter, or the point light) and a BSDF-sampled continuation;
//   emission is counted when a ray leaving a dielectric vertex hits the
//   quad emitter's front (paths next-event estimation cannot sample).
//   Uniforms: counter (s, 0, 2) film offsets; (s, j, 2) scattering
//   (u0, u1 direction, u2 dielectric lobe); (s, j, 3) the emitter point.
// Without spec_only the same tracer covers every path (the reference of
// the tests: its image equals the light tracer's plus the spec_only one).
struct CamTerm { V C[3]; };

double tent_offset(double xi) { return xi < 0.5 ? std::sqrt(2.0 * xi) - 1.0 : 1.0 - std::sqrt(2.0 - 2.0 * xi); }

// front-face hit of the quad emitter: t > 0 or -1, and its quad coordinates
double emitter_hit(const ora_scene& sc, D3 o, D3 d, double& a, double& b) {
  D3 O = {sc.em_o[0], sc.em_o[1], sc.em_o[2]}, e1 = {sc.em_e1[0], sc.em_e1[1], sc.em_e1[2]},
     e2 = {sc.em_e2[0], sc.em_e2[1], sc.em_e2[2]};
  D3 N = cross(e1, e2);
  double den = dot(d, N);
  if (!(den < 0.0)) return -1.0;
  double t = dot(O - o, N) / den;
  if (!(t > kTmin)) return -1.0;
  D3 q = o + d * t - O;
  double e11 = dot(e1, e1), e12 = dot(e1, e2), e22 = dot(e2, e2), q1 = dot(q, e1), q2 = dot(q, e2);
  double det = e11 * e22 - e12 * e12;
  a = (q1 * e22 - q2 * e12) / det; b = (q2 * e11 - q1 * e12) / det;
  if (a < 0.0 || a > 1.0 || b < 0.0 || b > 1.0) return -1.0;
  return t;
}

// emitter radiance leaves at quad coordinates (a, b)
void emitter_le(const Scene& S, double a, double b, V Le[3]) {
  const ora_scene& sc = *S.s;
  long le = 0;
  if (sc.em_tex_res > 0) {
    const int R = sc.em_tex_res;
    int tx = std::min((int)std::floor(a * R), R - 1), ty = std::min((int)std::floor(b * R), R - 1);
    le = 3L * ((long)ty * R + tx);
  }
  for (int c = 0; c < 3; ++c) Le[c] = leaf(S.Le[le + c], S.slot_Le + le + c);
}

// One camera sample: its pixel (-1 when the film offset leaves the film or
// the sample contributes nothing) and its estimator terms.
int camera_path(const Scene& S, const ora_args& A, uint32_t s, bool spec_only, std::vector<CamTerm>& terms,
                uint32_t& sig) {
  const ora_scene& sc = *S.s;
  const int W = sc.width, H = sc.height;
  terms.clear(); sig = 0x811C9DC5u;
  const uint32_t p = s % (uint32_t)(W * H);
  Uniform4 uf = rng4(A.seed, s, 0, 2);
  const double ux = (double)(p % W) + 0.5 + tent_offset(uf.u[0]), uy = (double)(p / W) + 0.5 + tent_offset(uf.u[1]);
  if (!(ux >= 0.0 && ux < W && uy >= 0.0 && uy < H)) return -1;
  const double qx = (2.0 * ux / W - 1.0) * S.aspect * S.tan_half, qy = (1.0 - 2.0 * uy / H) * S.tan_half;
  D3 d = normalize(S.f + S.r * qx + S.u * qy);
  D3 o = S.cpos;
  D3 offn = {0, 0, 0}; bool off = false, prev_spec = false;
  V beta[3] = {V(1.0), V(1.0), V(1.0)};
  const bool quad = sc.em_type == ORA_EMIT_QUAD;
  D3 eO = {sc.em_o[0], sc.em_o[1], sc.em_o[2]}, ee1 = {sc.em_e1[0], sc.em_e1[1], sc.em_e1[2]},
     ee2 = {sc.em_e2[0], sc.em_e2[1], sc.em_e2[2]};
  D3 eN = cross(ee1, ee2);
  const double earea = std::sqrt(dot(eN, eN));
  eN = eN * (1.0 / std::max(earea, 1e-300));
  for (int j = 1; j <= A.max_depth; ++j) {
    D3 xo = o;
    if (off) xo = xo + offn * (dot(d, offn) >= 0 ? kEps : -kEps);
    double th = 1e300;
    int tri = S.closest(xo, d, kTmin, 1e300, &th);
    if (quad && prev_spec) {  // emission seen through a specular chain
      double a, b;
      double te = emitter_hit(sc, xo, d, a, b);
      if (te > 0.0 && te <= th * (1.0 + 1e-9) + 1e-9) {
        V Le[3]; emitter_le(S, a, b, Le);
        CamTerm t; for (int c = 0; c < 3; ++c) t.C[c] = beta[c] * Le[c];
        terms.push_back(t);
        sig = fnv1a(sig, 0xE0u);  // the emitter is no occluder: the ray goes on
      }
    }
    if (tri < 0) { sig = fnv1a(sig, 0u); break; }
    sig = fnv1a(sig, (uint32_t)tri + 1u);
    int mat = S.mat_of(tri);
    int mtype = sc.mat_type[mat];
    if (mtype == ORA_ABSORBER) break;
    D3 x = xo + d * th;
    D3 P0 = S.tv[tri * 3], e1 = S.tv[tri * 3 + 1] - P0, e2 = S.tv[tri * 3 + 2] - P0;
    D3 Nn = cross(e1, e2);
    D3 ng = normalize(Nn);
    double nn = dot(Nn, Nn);
    D3 dx = x - P0;
    double b1 = dot(cross(dx, e2), Nn) / nn, b2 = dot(cross(e1, dx), Nn) / nn;
    const double cos_in = dot(d, ng);
    D3 ns = ng;
    if (tri >= S.n_static) {
      V sxv[3], szv[3];
      for (int k = 0; k < 3; ++k) { int gi, gj; S.hf_corner(tri, k, gi, gj); S.slope(gi, gj, sxv[k], szv[k]); }
      double c0 = 1.0 - b1 - b2;
      double Sx = c0 * sxv[0].v + b1 * sxv[1].v + b2 * sxv[2].v, Sz = c0 * szv[0].v + b1 * szv[1].v + b2 * szv[2].v;
      ns = normalize(D3{-Sx, 1.0, -Sz});
    }
    Uniform4 uj = rng4(A.seed, s, (uint32_t)j, 2);
    if (mtype == ORA_DIELECTRIC) {
      if (j == A.max_depth) break;
      V3 wo; bool reflect = false; double F = 0.0;
      int code = dielectric_event(cst(d), cst(ns), ng, sc.mat_ior[mat], uj.u[2], wo, reflect, F);
      if (code == 7) { sig = fnv1a(sig, 7u); break; }
      sig = fnv1a(sig, reflect ? 2u : 4u);
      if (code == 8) { sig = fnv1a(sig, 8u); break; }
      o = x; d = val(wo); offn = ng; off = true; prev_spec = true;
      continue;
    }
    if (spec_only && j == 1) return -1;  // the light tracer's paths
    // Lambertian or rough conductor: its texel, the arrival-side normal
    const bool cond = mtype == ORA_CONDUCTOR;
    int tex = sc.mat_tex[mat], R = sc.tex_res;
    double uvx = 0.0, uvy = 0.0;
    if (tri < S.n_static) {
      const double* uv = sc.tri_uv + (size_t)tri * 6;
      double c0 = 1.0 - b1 - b2;
      uvx = c0 * uv[0] + b1 * uv[2] + b2 * uv[4];
      uvy = c0 * uv[1] + b1 * uv[3] + b2 * uv[5];
    }
    int tx = std::min(std::max((int)std::floor(uvx * R), 0), R - 1), ty = std::min(std::max((int)std::floor(uvy * R), 0), R - 1);
    long texel = ((long)tex * R + ty) * R + tx;
    sig = fnv1a(sig, (uint32_t)texel + 1u);
    V rho[3];
    for (int c = 0; c < 3; ++c) rho[c] = leaf(S.albedo[texel * 3 + c], texel * 3 + c);
    const D3 na = cond ? (cos_in < 0 ? ns : ns * -1.0) : (cos_in < 0 ? ng : ng * -1.0);
    const D3 wv = d * -1.0;  // toward the camera side
    if (cond && !(dot(wv, na) > 0.0)) { sig = fnv1a(sig, 9u); break; }
    // --- next-event estimation
    {
      Uniform4 ue = rng4(A.seed, s, (uint32_t)j, 3);
      D3 y; double geo; V Le[3];
      if (quad) {
        y = eO + ee1 * ue.u[0] + ee2 * ue.u[1];
        emitter_le(S, ue.u[0], ue.u[1], Le);
      } else {
        y = eO;
        for (int c = 0; c < 3; ++c) Le[c] = leaf(S.Le[c], S.slot_Le + c);
      }
      D3 dl = y - x;
      double r2 = dot(dl, dl), r = std::sqrt(r2);
      D3 wl = dl * (1.0 / r);
      double cy = quad ? -dot(wl, eN) : 1.0;
      double cx = dot(wl, na), cg = dot(wl, ng) * (cos_in < 0 ? 1.0 : -1.0);
      uint32_t vis = 0;
      if (cy > 0.0 && cx > 0.0 && cg > 0.0) {
        D3 so = x + ng * (dot(wl, ng) >= 0 ? kEps : -kEps);
        D3 sd = y - so;
        double sl = std::sqrt(dot(sd, sd));
        if (S.closest(so, sd * (1.0 / sl), kTmin, sl * (1.0 - 1e-4), nullptr) < 0) {
          vis = 1;
          geo = quad ? cy * earea / r2 : 1.0 / r2;
          double fb;  // f cos_x / rho
          if (!cond) fb = kInvPi * cx;
          else {
            // conductor: f(wv, wl) (wl.na) / F0 = D G1 G1 / (4 wv.na)
            fb = conductor_conn(cst(wv), cst(wl), cst(na), sc.mat_ior[mat]).v;
          }
          CamTerm t;
          for (int c = 0; c < 3; ++c) t.C[c] = beta[c] * rho[c] * Le[c] * V(fb * geo);
          terms.push_back(t);
        }
      }
      sig = fnv1a(sig, vis);
    }
    if (j == A.max_depth) break;
    // --- BSDF-sampled continuation
    if (cond) {
      V3 wo; V wgt;
      int code = conductor_event(cst(wv), cst(na), ng, cos_in < 0 ? 1.0 : -1.0, sc.mat_ior[mat], uj.u[0], uj.u[1], wo, wgt);
      if (code) { sig = fnv1a(sig, (uint32_t)code); break; }
      for (int c = 0; c < 3; ++c) beta[c] = beta[c] * rho[c] * V(wgt.v);
      d = val(wo);
    } else {
      double rr = std::sqrt(uj.u[0]), phi = 2.0 * M_PI * uj.u[1];
      D3 t1, t2; onb(na, t1, t2);
      d = t1 * (rr * std::cos(phi)) + t2 * (rr * std::sin(phi)) + na * std::sqrt(std::max(0.0, 1.0 - uj.u[0]));
      for (int c = 0; c < 3; ++c) beta[c] = beta[c] * rho[c];
    }
    o = x; offn = ng; off = true; prev_spec = false;
  }
  return terms.empty() ? -1 : (int)p;
}

// tent filter taps (radius 1 pixel, taps outside the film dropped)
struct Tap { int px, py; V w; };
int taps(const Conn& cn, int W, int H, Tap t[4]) {
  int px0 = (int)std::floor(cn.ux.v - 0.5), py0 = (int)std::floor(cn.uy.v - 0.5);
  int n = 0;
  for (int dy = 0; dy < 2; ++dy)
    for (int dx = 0; dx < 2; ++dx) {
      int px = px0 + dx, py = py0 + dy;
      if (px < 0 || px >= W || py < 0 || py >= H) continue;
      V wx = V(1.0) - vabs(cn.ux - V(px + 0.5));
      V wy = V(1.0) - vabs(cn.uy - V(py + 0.5));
      t[n++] = {px, py, wx * wy};
    }
  return n;
}

}  // namespace

extern "C" {

int ora_version() { return 1; }

// u = (philox(...) >> 8) * 2^-24 for external known-answer checks.
void ora_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t* out) {
  U4 c{{c0, c1, c2, c3}};
  U4 r = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  for (int i = 0; i < 4; ++i) out[i] = r.x[i];
}

// Weighted reservoir of capacity one over a candidate stream (Eq. 8):
// returns the 1-based selected index (0 if every weight is zero).
int ora_reservoir(const double* w, const double* u, int k, double* W_out) {
  double Om = 0.0, wr = 0.0; int R = 0;
  for (int i = 0; i < k; ++i) {
    if (!(w[i] > 0.0)) continue;
    Om += w[i];
    if (u[i] < w[i] / Om) { R = i + 1; wr = w[i]; }
  }
  if (W_out) *W_out = R ? Om / wr : 0.0;
  return R;
}

// GGX terms at roughness a: D(m) for m.n = cm and G1 for v.n = cv.
void ora_ggx_terms(double a, double cm, double cv, double* D, double* G1) {
  *D = ggx_D(V(cm), a * a).v;
  *G1 = ggx_G1(V(cv), a * a).v;
}

// One rough-conductor reflection with constant inputs (wi, n unit, wi on the
// side of n; ng = n): writes wo and the weight f (wo.n) / p over F0.  Returns
// the event code of conductor_event.
int ora_conductor(const double* wi, const double* n, double a, double u0, double u1, double* wo, double* wgt) {
  V3 w = cst({wi[0], wi[1], wi[2]}), nn = cst({n[0], n[1], n[2]});
  V3 o{V(0.0), V(0.0), V(0.0)};
  V g(0.0);
  int code = conductor_event(w, nn, {n[0], n[1], n[2]}, 1.0, a, u0, u1, o, g);
  wo[0] = o.x.v; wo[1] = o.y.v; wo[2] = o.z.v;
  *wgt = g.v;
  return code;
}

// The conductor's connection factor f (wc.n) / F0 for constant unit wi, wc, n.
double ora_conductor_conn(const double* wi, const double* wc, const double* n, double a) {
  return conductor_conn(cst({wi[0], wi[1], wi[2]}), cst({wc[0], wc[1], wc[2]}), cst({n[0], n[1], n[2]}), a).v;
}

// One dielectric scattering event with constant inputs (w_in, ng, ns unit
// 3-vectors; ns on the side of ng): writes the new direction wo (when the
// return value is 0 or 8), whether the reflection lobe was taken and the
// Fresnel reflectance F.  Returns the event code of dielectric_event.
int ora_dielectric(const double* w_in, const double* ng, const double* ns, double ior, double u_lobe, double* wo,
                   int32_t* reflect, double* F) {
  V3 w = cst({w_in[0], w_in[1], w_in[2]}), n = cst({ns[0], ns[1], ns[2]});
  V3 o;
  bool refl = false;
  double f = 0.0;
  int code = dielectric_event(w, n, {ng[0], ng[1], ng[2]}, ior, u_lobe, o, refl, f);
  if (code != 7) { wo[0] = o.x.v; wo[1] = o.y.v; wo[2] = o.z.v; }
  if (reflect) *reflect = refl ? 1 : 0;
  if (F) *F = f;
  return code;
}

// Forward render.  image: [H][W][3] (overwritten).  Optional outputs:
// slices [D][H][W][3] (connections of vertex i land in slice i-1),
// sig/R/Wres per listed path, flux = sum over connections of C (3 doubles),
// info per listed path (bit 1: an ill-conditioned vertex at or before the
// last sensor connection, see PathResult; bit 2: a guided scatter from an
// entry marked in guide_flag).
int ora_render(const ora_scene* sc, const ora_args* A, const double* albedo, const double* Le,
               const double* heights, const double* nmap, double* image, double* slices, uint32_t* sig,
               int32_t* Rout, double* Wout, double* flux, uint32_t* info) {
  if (A->guide_w && sc->em_type != ORA_EMIT_QUAD) return -1;  // the guide steers area emission only
  if (sc->em_tex_res > 0 && sc->em_type == ORA_EMIT_POINT) return -1;
  Scene S; S.init(sc, albedo, Le, heights, nmap, false);
  if (A->guide_w && A->guide_diffuse) build_guide_table(S, *A, nullptr);
  const int W = sc->width, H = sc->height, D = A->max_depth;
  const long npix = (long)W * H * 3;
  const int64_t n = A->path_list ? A->n_list : A->n_paths;
  int nt = A->n_threads > 0 ? A->n_threads : omp_get_max_threads();
  std::vector<std::vector<double>> img(nt, std::vector<double>(npix, 0.0));
  std::vector<std::vector<double>> sl(slices ? nt : 0, std::vector<double>(slices ? npix * D : 0, 0.0));
  std::vector<double> fl((size_t)nt * 3, 0.0);
  const bool selected = (A->flags & ORA_F_SPLAT_SELECTED) != 0;
#pragma omp parallel num_threads(nt)
  {
    int tid = omp_get_thread_num();
    Tape tape; g_tape = &tape;
    PathResult pr;
#pragma omp for schedule(dynamic, 256)
    for (int64_t k = 0; k < n; ++k) {
      uint32_t path = A->path_list ? A->path_list[k] : (uint32_t)k;
      tape.clear();
      trace_path(S, *A, path, pr);
      if (sig) sig[k] = pr.sig;
      if (Rout) Rout[k] = pr.R;
      if (Wout) Wout[k] = pr.W;
      if (info) info[k] = (pr.illc ? 2u : 0u) | (pr.gflag ? 4u : 0u);
      for (size_t ci = 0; ci < pr.conns.size(); ++ci) {
        const Conn& cn = pr.conns[ci];
        double scale = 1.0;
        if (selected) { if (cn.depth != pr.R) continue; scale = pr.W; }
        for (int c = 0; c < 3; ++c) fl[tid * 3 + c] += scale * cn.C[c].v;
        Tap t[4]; int nt4 = taps(cn, W, H, t);
        for (int q = 0; q < nt4; ++q) {
          long p = ((long)t[q].py * W + t[q].px) * 3;
          for (int c = 0; c < 3; ++c) {
            double v = scale * t[q].w.v * cn.C[c].v;
            img[tid][p + c] += v;
            if (slices) sl[tid][(long)(cn.depth - 1) * npix + p + c] += v;
          }
        }
      }
    }
    g_tape = nullptr;
  }
  for (long p = 0; p < npix; ++p) { double s = 0; for (int t = 0; t < nt; ++t) s += img[t][p]; image[p] = s; }
  if (slices)
    for (long p = 0; p < npix * D; ++p) { double s = 0; for (int t = 0; t < nt; ++t) s += sl[t][p]; slices[p] = s; }
  if (flux) for (int c = 0; c < 3; ++c) { double s = 0; for (int t = 0; t < nt; ++t) s += fl[t * 3 + c]; flux[c] = s; }
  return 0;
}

// Camera-side image (see camera_path): image [H][W][3] (overwritten) from
// the listed camera samples (A->path_list, else [0, n_paths)); each pixel
// averages spp = n_paths / (W H) samples (n_paths a multiple of W H).
// spec_only 1: only samples whose first vertex is specular.  sig per listed
// sample when given.  Returns -1 for an emitter the camera cannot sample
// (directional) or n_paths not a multiple of W H.
int ora_render_camera(const ora_scene* sc, const ora_args* A, int spec_only, const double* albedo, const double* Le,
                      const double* heights, const double* nmap, double* image, uint32_t* sig) {
  const long npx = (long)sc->width * sc->height;
  if (sc->em_type == ORA_EMIT_DIRECTIONAL || A->n_paths % npx != 0) return -1;
  Scene S; S.init(sc, albedo, Le, heights, nmap, false);
  const double inv_spp = (double)npx / (double)A->n_paths;
  const int64_t n = A->path_list ? A->n_list : A->n_paths;
  int nt = A->n_threads > 0 ? A->n_threads : omp_get_max_threads();
  std::vector<std::vector<double>> img(nt, std::vector<double>(npx * 3, 0.0));
#pragma omp parallel num_threads(nt)
  {
    int tid = omp_get_thread_num();
    Tape tape; g_tape = &tape;
    std::vector<CamTerm> terms;
#pragma omp for schedule(dynamic, 256)
    for (int64_t k = 0; k < n; ++k) {
      uint32_t smp = A->path_list ? A->path_list[k] : (uint32_t)k;
      tape.clear();
      uint32_t sg;
      int px = camera_path(S, *A, smp, spec_only != 0, terms, sg);
      if (sig) sig[k] = sg;
      if (px < 0) continue;
      for (const CamTerm& t : terms)
        for (int c = 0; c < 3; ++c) img[tid][px * 3 + c] += inv_spp * t.C[c].v;
    }
    g_tape = nullptr;
  }
  for (long q = 0; q < npx * 3; ++q) { double v = 0; for (int t = 0; t < nt; ++t) v += img[t][q]; image[q] = v; }
  return 0;
}

// Gradient of <dI, I_camera> w.r.t. albedo texels and emitter radiance
// (detached) by taped reverse-mode AD of each camera sample; accumulated.
int ora_gradient_camera(const ora_scene* sc, const ora_args* A, int spec_only, const double* albedo, const double* Le,
                        const double* heights, const double* nmap, const double* dI, double* g_albedo, double* g_Le) {
  const long npx = (long)sc->width * sc->height;
  if (sc->em_type == ORA_EMIT_DIRECTIONAL || A->n_paths % npx != 0) return -1;
  Scene S; S.init(sc, albedo, Le, heights, nmap, false);
  const double inv_spp = (double)npx / (double)A->n_paths;
  const int64_t n = A->path_list ? A->n_list : A->n_paths;
  const long n_alb = S.slot_Le, nslot = n_alb + S.n_le;
  int nt = A->n_threads > 0 ? A->n_threads : omp_get_max_threads();
  std::vector<std::vector<double>> gr(nt, std::vector<double>(nslot, 0.0));
#pragma omp parallel num_threads(nt)
  {
    int tid = omp_get_thread_num();
    Tape tape; g_tape = &tape;
    std::vector<CamTerm> terms;
    std::vector<double> adj;
#pragma omp for schedule(dynamic, 256)
    for (int64_t k = 0; k < n; ++k) {
      uint32_t smp = A->path_list ? A->path_list[k] : (uint32_t)k;
      tape.clear();
      uint32_t sg;
      int px = camera_path(S, *A, smp, spec_only != 0, terms, sg);
      if (px < 0) continue;
      V lam(0.0);
      for (const CamTerm& t : terms)
        for (int c = 0; c < 3; ++c) lam = lam + t.C[c] * V(inv_spp * dI[px * 3 + c]);
      if (lam.i < 0) continue;
      adj.assign(tape.a.size(), 0.0);
      adj[lam.i] = 1.0;
      for (int q = lam.i; q >= 0; --q) {
        double g = adj[q];
        if (g == 0.0) continue;
        if (tape.a[q] >= 0) adj[tape.a[q]] += g * tape.da[q];
        if (tape.b[q] >= 0) adj[tape.b[q]] += g * tape.db[q];
      }
      for (auto& lf : tape.leaves) if (lf.second < nslot) gr[tid][lf.second] += adj[lf.first];
    }
    g_tape = nullptr;
  }
  for (long q = 0; q < nslot; ++q) {
    double v = 0; for (int t = 0; t < nt; ++t) v += gr[t][q];
    if (q < n_alb) { if (g_albedo) g_albedo[q] += v; }
    else if (g_Le) g_Le[q - n_alb] += v;
  }
  return 0;
}

// Gradient of <dI, I(theta)> (= dLoss/dtheta when dI = dLoss/dI) by taped
// reverse-mode AD of each path.  mode NAIVE: every connection;
// mode RESLRB: only the reservoir-selected connection, scaled by the fixed
// weight Omega_k/omega_R (Eq. 11).  Gradients are accumulated into g_*
// (g_heights only when ORA_F_ATTACHED and the scene has a heightfield).
int ora_gradient(const ora_scene* sc, const ora_args* A, int mode, const double* albedo,
                 const double* Le, const double* heights, const double* nmap, const double* dI, double* g_albedo,
                 double* g_Le, double* g_heights, double* g_nmap) {
  if (A->guide_w && sc->em_type != ORA_EMIT_QUAD) return -1;
  if (sc->em_tex_res > 0 && sc->em_type == ORA_EMIT_POINT) return -1;
  Scene S; S.init(sc, albedo, Le, heights, nmap, (A->flags & ORA_F_ATTACHED) != 0);
  if (A->guide_w && A->guide_diffuse) build_guide_table(S, *A, nullptr);
  const int W = sc->width, H = sc->height;
  const int64_t n = A->path_list ? A->n_list : A->n_paths;
  const long n_alb = S.slot_Le, n_h = sc->hf_G > 1 ? (long)sc->hf_G * sc->hf_G : 0;
  const long n_n = S.nmap ? 2 * n_h : 0, n_le = S.n_le;
  const long nslot = n_alb + n_le + n_h + n_n;
  int nt = A->n_threads > 0 ? A->n_threads : omp_get_max_threads();
  std::vector<std::vector<double>> gr(nt, std::vector<double>(nslot, 0.0));
#pragma omp parallel num_threads(nt)
  {
    int tid = omp_get_thread_num();
    Tape tape; g_tape = &tape;
    PathResult pr;
    std::vector<double> adj;
#pragma omp for schedule(dynamic, 256)
    for (int64_t k = 0; k < n; ++k) {
      uint32_t path = A->path_list ? A->path_list[k] : (uint32_t)k;
      tape.clear();
      trace_path(S, *A, path, pr);
      // scalar objective lambda = sum_i sum_taps F(u_i,p) <dI[p], C_i>
      V lam(0.0);
      for (size_t ci = 0; ci < pr.conns.size(); ++ci) {
        const Conn& cn = pr.conns[ci];
        if (mode == ORA_MODE_RESLRB && cn.depth != pr.R) continue;
        Tap t[4]; int nt4 = taps(cn, W, H, t);
        V term(0.0);
        for (int q = 0; q < nt4; ++q) {
          long p = ((long)t[q].py * W + t[q].px) * 3;
          V inner = cn.C[0] * V(dI[p]) + cn.C[1] * V(dI[p + 1]) + cn.C[2] * V(dI[p + 2]);
          term = term + t[q].w * inner;
        }
        if (mode == ORA_MODE_RESLRB) term = term * V(pr.W);
        lam = lam + term;
      }
      if (lam.i < 0) continue;
      adj.assign(tape.a.size(), 0.0);
      adj[lam.i] = 1.0;
      for (int q = lam.i; q >= 0; --q) {
        double g = adj[q];
        if (g == 0.0) continue;
        if (tape.a[q] >= 0) adj[tape.a[q]] += g * tape.da[q];
        if (tape.b[q] >= 0) adj[tape.b[q]] += g * tape.db[q];
      }
      for (auto& lf : tape.leaves) gr[tid][lf.second] += adj[lf.first];
    }
    g_tape = nullptr;
  }
  for (long q = 0; q < nslot; ++q) {
    double s = 0; for (int t = 0; t < nt; ++t) s += gr[t][q];
    if (q < n_alb) { if (g_albedo) g_albedo[q] += s; }
    else if (q < n_alb + n_le) { if (g_Le) g_Le[q - n_alb] += s; }
    else if (q < n_alb + n_le + n_h) { if (g_heights) g_heights[q - n_alb - n_le] += s; }
    else if (g_nmap) g_nmap[q - n_alb - n_le - n_h] += s;
  }
  return 0;
}

// ----------------------------------------------------------------- guide API
int ora_guide_nparams() { return (int)kGN; }

// Raw network outputs [count][41] for positions x and unit normals n [count][3].
int ora_guide_eval(const ora_scene* sc, const double* w, const double* x, const double* n, int64_t count,
                   int bf16, double* out) {
  double c[3], h[3]; scene_box(sc, c, h);
  for (int64_t i = 0; i < count; ++i) {
    double f[kGIn];
    guide_features(c, h, {x[i * 3], x[i * 3 + 1], x[i * 3 + 2]}, {n[i * 3], n[i * 3 + 1], n[i * 3 + 2]}, f);
    GuideAct a; guide_forward(w, f, bf16 != 0, a);
    for (int k = 0; k < kGOut; ++k) out[i * kGOut + k] = a.o[k];
  }
  return 0;
}

// Folded mixture density of raw outputs o [count][41] at directions wd.
int ora_guide_pdf(const double* o, const double* n, const double* wd, int64_t count, double* pdf) {
  for (int64_t i = 0; i < count; ++i) {
    Mixture m = mixture_of(o + i * kGOut);
    pdf[i] = guide_pdf(m, {n[i * 3], n[i * 3 + 1], n[i * 3 + 2]}, {wd[i * 3], wd[i * 3 + 1], wd[i * 3 + 2]});
  }
  return 0;
}

// Directions drawn from raw outputs o with uniforms g [count][3].
int ora_guide_sample(const double* o, const double* n, const double* g, int64_t count, double* wd, int32_t* comp) {
  for (int64_t i = 0; i < count; ++i) {
    Mixture m = mixture_of(o + i * kGOut);
    int cp;
    D3 w = guide_sample(m, {n[i * 3], n[i * 3 + 1], n[i * 3 + 2]}, g[i * 3], g[i * 3 + 1], g[i * 3 + 2], cp);
    wd[i * 3] = w.x; wd[i * 3 + 1] = w.y; wd[i * 3 + 2] = w.z;
    if (comp) comp[i] = cp;
  }
  return 0;
}

// Guide table (see build_guide_table): raw network outputs per entry
// raw [2 T][41], texel centres x, n [T][3] and coverage ok [T], T the number
// of albedo texels.  Returns T, or -1 without guide weights.
int64_t ora_guide_table(const ora_scene* sc, const ora_args* A, double* raw, double* x, double* n, uint8_t* ok) {
  if (!A->guide_w) return -1;
  Scene S; S.init(sc, nullptr, nullptr, nullptr, nullptr, false);
  std::vector<double> r, xv, nv; std::vector<uint8_t> okv;
  texel_centres(sc, xv, nv, okv);
  build_guide_table(S, *A, &r);
  const int64_t T = (int64_t)okv.size();
  if (raw) std::copy(r.begin(), r.end(), raw);
  if (x) std::copy(xv.begin(), xv.end(), x);
  if (n) std::copy(nv.begin(), nv.end(), n);
  if (ok) std::copy(okv.begin(), okv.end(), ok);
  return T;
}

// Training samples of the diffuse guide, one per listed path: the path's
// first guided Lambertian scatter (position, arrival-side normal, sampled
// direction, density q, component) with S = sum of lum(C_i) over the path's
// connections after that vertex (the contribution the direction carried),
// in the 12-double layout of ora_guide_emit's samples; all zero for a path
// with no guided scatter.  Needs guide_w and guide_diffuse.
int ora_guide_vertex_samples(const ora_scene* sc, const ora_args* A, const double* albedo, const double* Le,
                             const double* heights, const double* nmap, double* out) {
  if (!A->guide_w || !A->guide_diffuse || sc->em_type != ORA_EMIT_QUAD) return -1;
  Scene S; S.init(sc, albedo, Le, heights, nmap, false);
  build_guide_table(S, *A, nullptr);
  const int64_t n = A->path_list ? A->n_list : A->n_paths;
  int nt = A->n_threads > 0 ? A->n_threads : omp_get_max_threads();
#pragma omp parallel num_threads(nt)
  {
    Tape tape; g_tape = &tape;
    PathResult pr;
#pragma omp for schedule(dynamic, 256)
    for (int64_t k = 0; k < n; ++k) {
      uint32_t path = A->path_list ? A->path_list[k] : (uint32_t)k;
      tape.clear();
      trace_path(S, *A, path, pr);
      double* o = out + k * 12;
      for (int q = 0; q < 12; ++q) o[q] = 0.0;
      if (!pr.gdepth) continue;
      double Sd = 0.0;
      for (const Conn& cn : pr.conns)
        if (cn.depth > pr.gdepth) Sd += kLumR * cn.C[0].v + kLumG * cn.C[1].v + kLumB * cn.C[2].v;
      for (int q = 0; q < 3; ++q) { o[q] = pr.gx[q]; o[3 + q] = pr.gn[q]; o[6 + q] = pr.gwd[q]; }
      o[9] = pr.gq; o[10] = Sd; o[11] = pr.gcomp;
    }
    g_tape = nullptr;
  }
  return 0;
}

// Guided emission samples of the listed paths (A->path_list, else [0, n_paths)):
// rec [n][8] = position x0 (3), direction (3), density q, emission factor
// A cos / q (beta_1 = L_e * factor); comp [n] as in ora_guide_sample.
int ora_guide_emit(const ora_scene* sc, const ora_args* A, double* rec, int32_t* comp) {
  if (!A->guide_w || sc->em_type != ORA_EMIT_QUAD) return -1;
  double c[3], h[3]; scene_box(sc, c, h);
  D3 o = {sc->em_o[0], sc->em_o[1], sc->em_o[2]};
  D3 e1 = {sc->em_e1[0], sc->em_e1[1], sc->em_e1[2]}, e2 = {sc->em_e2[0], sc->em_e2[1], sc->em_e2[2]};
  D3 cr = cross(e1, e2);
  double area = std::sqrt(dot(cr, cr));
  D3 ne = cr * (1.0 / area);
  const int64_t n = A->path_list ? A->n_list : A->n_paths;
  for (int64_t k = 0; k < n; ++k) {
    uint32_t path = A->path_list ? A->path_list[k] : (uint32_t)k;
    Uniform4 u0 = rng4(A->seed, path, 0, 0);
    D3 x0 = o + e1 * u0.u[0] + e2 * u0.u[1];
    double f[kGIn]; guide_features(c, h, x0, ne, f);
    GuideAct a; guide_forward(A->guide_w, f, A->guide_bf16 != 0, a);
    Mixture m = mixture_of(a.o);
    Uniform4 g = rng4(A->seed, path, 0, 1);
    int cp;
    D3 w = guide_sample(m, ne, g.u[0], g.u[1], g.u[2], cp);
    double q = guide_pdf(m, ne, w);
    double* r = rec + k * 8;
    r[0] = x0.x; r[1] = x0.y; r[2] = x0.z; r[3] = w.x; r[4] = w.y; r[5] = w.z;
    r[6] = q; r[7] = q > 0.0 ? area * dot(w, ne) / q : 0.0;
    if (comp) comp[k] = cp;
  }
  return 0;
}

// Training loss L = -sum_b (S_b / q_b) log q_theta(w_b | x_b, n_b) / Z, with
// Z = sum_b S_b / q_b (self-normalised, so the scale of S does not matter),
// and its gradient w.r.t. the parameters (added to grad [11433]); zero when
// Z is.  samples [count][12] = x (3), n (3), w (3), q (sampling density), S, unused.
int ora_guide_loss_grad(const ora_scene* sc, const double* w, const double* samples, int64_t count, int bf16,
                        double* grad, double* loss) {
  double c[3], h[3]; scene_box(sc, c, h);
  double Z = 0.0;
  for (int64_t b = 0; b < count; ++b) {
    const double* s = samples + b * 12;
    if (s[9] > 0.0 && s[10] != 0.0) Z += s[10] / s[9];
  }
  double L = 0.0;
  for (int64_t b = 0; b < count; ++b) {
    const double* s = samples + b * 12;
    double qs = s[9], S = s[10];
    if (!(qs > 0.0) || S == 0.0 || !(Z > 0.0)) continue;
    double f[kGIn];
    D3 nn = {s[3], s[4], s[5]};
    guide_features(c, h, {s[0], s[1], s[2]}, nn, f);
    GuideAct a; guide_forward(w, f, bf16 != 0, a);
    double go[kGOut];
    L += guide_loss_grad_o(a.o, nn, {s[6], s[7], s[8]}, S / (qs * Z), go);
    guide_backward(w, a, go, bf16 != 0, grad);
  }
  if (loss) *loss = L;
  return 0;
}

}  // extern "C"
