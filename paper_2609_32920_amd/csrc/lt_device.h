// Device-side building blocks of the light tracer (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "lt_common.h"

namespace lt {

// Diagnostic event counters, compiled only into the LT_COUNTERS build:
// 0 closest-hit rays, 1 shadow rays, 2 BVH node fetches, 3 triangle tests,
// 4 film splats, 5 adjoint gathers, 6 gradient values scattered,
// 7 paths emitted, 8 tape records written, 9 tape records read.
// Translation units without counted events define LT_NO_EVENT_COUNTERS so
// that the counter array has a single definition.
#if defined(LT_COUNTERS) && !defined(LT_NO_EVENT_COUNTERS)
__device__ unsigned long long lt_counters[16];
#define LT_COUNT(k, v) atomicAdd(&lt_counters[k], (unsigned long long)(v))
#else
#define LT_COUNT(k, v) ((void)0)
#endif

// ------------------------------------------------------------ vector math
struct f3 { float x, y, z; };
__device__ __forceinline__ f3 mk(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ f3 ld3(const float* p) { return {p[0], p[1], p[2]}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ f3 mul(f3 a, f3 b) { return {a.x * b.x, a.y * b.y, a.z * b.z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross(f3 a, f3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ f3 normalize(f3 a) { return a * (1.0f / sqrtf(dot(a, a))); }

// ------------------------------------------------------------ Philox RNG
// Philox-4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed with
// counter (path, vertex, block, 0); outputs become 24-bit uniforms in [0,1).
struct u4f { float u0, u1, u2, u3; };

__device__ __forceinline__ u4f rng4(uint64_t seed, uint32_t path, uint32_t vtx, uint32_t block) {
  uint32_t c0 = path, c1 = vtx, c2 = block, c3 = 0u;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  const float s = 5.9604644775390625e-8f;  // 2^-24
  return {(float)(c0 >> 8) * s, (float)(c1 >> 8) * s, (float)(c2 >> 8) * s, (float)(c3 >> 8) * s};
}

__device__ __forceinline__ uint32_t fnv1a(uint32_t h, uint32_t w) {
#pragma unroll
  for (int b = 0; b < 4; ++b) { h ^= (w >> (8 * b)) & 0xFFu; h *= 0x01000193u; }
  return h;
}

// Orthonormal basis around unit n (Duff et al., JCGT 2017).
__device__ __forceinline__ void onb(f3 n, f3& b1, f3& b2) {
  float sign = copysignf(1.0f, n.z);
  float a = -1.0f / (sign + n.z);
  float b = n.x * n.y * a;
  b1 = {1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x};
  b2 = {b, sign + n.y * n.y * a, -n.y};
}

// cosine-weighted direction about n (Malley's method) from (u0, u1)
__device__ __forceinline__ f3 cosine_dir(f3 n, float u0, float u1) {
  // sin/cos of 2*pi*u1 via sinpi/cospi: 2*u1 is exact, so no rounding of
  // the angle itself enters the direction
  float r = sqrtf(u0);
  float s = sinpif(2.0f * u1), c = cospif(2.0f * u1);
  f3 t1, t2; onb(n, t1, t2);
  float lz = sqrtf(fmaxf(0.0f, 1.0f - u0));
  return t1 * (r * c) + t2 * (r * s) + n * lz;
}

// von Mises-Fisher direction about the unit mean mu (concentration kap,
// em = 1 - e^{-2 kap}) from (g1, g2): the cosine t to mu by inverting its
// marginal (Wood 1994; Jakob 2012), 1 - t = -log(1 - g1 em) / kap, and
// sin^2 = (1 - t)(1 + t), so there is no cancellation near the mean.
__device__ __forceinline__ f3 vmf_dir(f3 mu, float kap, float em, float g1, float g2) {
  float u = -log1pf(-g1 * em) / kap;
  u = fminf(fmaxf(u, 0.0f), 2.0f);
  float t = 1.0f - u;
  float s = sqrtf(u * (2.0f - u));
  float sp = sinpif(2.0f * g2), cp = cospif(2.0f * g2);
  f3 t1, t2; onb(mu, t1, t2);
  return mu * t + t1 * (s * cp) + t2 * (s * sp);
}

// ------------------------------------------------------------ rough conductor
// GGX (Trowbridge-Reitz) microfacets of roughness a about the unit normal n,
// Smith's separable masking, reflectance F0 (the material's texel, constant
// in angle):  D(m) = a^2 / (pi ((m.n)^2 (a^2 - 1) + 1)^2),
// G1(v) = 2 (v.n) / ((v.n) + sqrt(a^2 + (1 - a^2)(v.n)^2)),
// f = F0 D(h) G1(wi) G1(wo) / (4 (wi.n)(wo.n)).
__device__ __forceinline__ float ggx_D(float cm, float a2) {
  float d = cm * cm * (a2 - 1.0f) + 1.0f;
  return a2 * 0.318309886183790672f / (d * d);
}
__device__ __forceinline__ float ggx_G1(float cv, float a2) { return 2.0f * cv / (cv + sqrtf(a2 + (1.0f - a2) * cv * cv)); }

// f (wc.n) / F0 = D(h) G1(wi) G1(wc) / (4 wi.n) of a sensor connection
__device__ __forceinline__ float ggx_conn(f3 wi, f3 wc, f3 n, float a) {
  const float a2 = a * a;
  f3 h = normalize(wi + wc);
  float ci = dot(wi, n);
  return ggx_D(dot(h, n), a2) * ggx_G1(ci, a2) * ggx_G1(dot(wc, n), a2) / (4.0f * ci);
}

// Local microfacet normal drawn with density D(m)(m.n) from (u0, u1):
// tan^2 theta = a^2 u0 / (1 - u0), phi = 2 pi u1.
__device__ __forceinline__ void ggx_local(float a, float u0, float u1, float& lx, float& ly, float& lz) {
  float t2 = a * a * u0 / (1.0f - u0);
  lz = 1.0f / sqrtf(1.0f + t2);
  float st = sqrtf(t2) * lz;
  lx = st * cospif(2.0f * u1);
  ly = st * sinpif(2.0f * u1);
}

// Reflection of wi (unit, away from the surface, wi.n > 0) about the drawn
// microfacet normal held in the local frame of n: wo and the weight
// f (wo.n) / p over F0 = G1(wi) G1(wo) (wi.m) / ((wi.n)(m.n)).  Returns 7
// when wi does not see the microfacet, 8 when wo leaves below n or on the
// far side of the geometric normal ng (side_in = +1: arrived on the +ng
// side), else 0.
__device__ __forceinline__ int conductor_scatter(f3 wi, f3 n, f3 ng, float side_in, float a, float u0, float u1,
                                                 f3& wo, float& wgt) {
  float lx, ly, lz;
  ggx_local(a, u0, u1, lx, ly, lz);
  f3 t1, t2; onb(n, t1, t2);
  f3 m = t1 * lx + t2 * ly + n * lz;
  float cwm = dot(wi, m);
  if (!(cwm > 0.0f)) return 7;
  wo = m * (2.0f * cwm) - wi;
  float co = dot(wo, n);
  if (!(co > 0.0f) || !(dot(wo, ng) * side_in > 0.0f)) return 8;
  const float a2 = a * a, ci = dot(wi, n);
  wgt = ggx_G1(ci, a2) * ggx_G1(co, a2) * cwm / (ci * lz);
  return 0;
}

// ------------------------------------------------------------ diffuse guide
// A guide-table entry: the folded vMF mixture of the learned guide at one
// side of one albedo texel, 16 float4.  Lobe k: [2k] = (mean direction,
// kappa), [2k+1] = (mixture weight, vMF normaliser kappa / (2 pi em),
// em = 1 - e^{-2 kappa}, the mixing weight alpha for k = 0).  alpha < 0
// marks an entry without a guide: the vertex samples the cosine density.
// Density about the unit arrival-side normal n:
//   q(w) = alpha sum_k pi_k [v_k(w) + v_k(mirror(w))] + (1 - alpha) max(w.n, 0) / pi.
constexpr int kGTabLobes = 8;

__device__ __forceinline__ float gtab_pdf(const float4* e, f3 n, f3 w) {
  float c = dot(w, n);
  if (c < 0.f) return 0.f;
  f3 wm = w - n * (2.0f * c);
  float V = 0.f;
#pragma unroll
  for (int k = 0; k < kGTabLobes; ++k) {
    float4 a = e[2 * k], b = e[2 * k + 1];
    f3 mu = {a.x, a.y, a.z};
    V += b.x * b.y * (expf(a.w * (dot(mu, w) - 1.0f)) + expf(a.w * (dot(mu, wm) - 1.0f)));
  }
  float al = e[1].w;
  return al * V + (1.0f - al) * c * 0.318309886183790672f;
}

// Draw from entry e about n: the component by g0 (cosine when g0 >= alpha,
// else the lobe whose cumulative weight first exceeds g0 / alpha), the
// direction by (g1, g2), a lobe direction below the surface mirrored
// about it.  Returns the direction, its density q and the component
// (0 cosine, k + 1 lobe k).
__device__ __forceinline__ f3 gtab_sample(const float4* e, f3 n, float g0, float g1, float g2, float& q,
                                           int& comp) {
  const float al = e[1].w;
  f3 w;
  comp = 0;
  if (g0 >= al) {
    w = cosine_dir(n, g1, g2);
  } else {
    float v = g0 / al, acc = 0.f;
    int k = kGTabLobes - 1;
#pragma unroll
    for (int i = 0; i < kGTabLobes; ++i) {
      acc += e[2 * i + 1].x;
      if (v < acc) { k = i; break; }
    }
    comp = k + 1;
    float4 a = e[2 * k], b = e[2 * k + 1];
    w = vmf_dir(mk(a.x, a.y, a.z), a.w, b.z, g1, g2);
    float c = dot(w, n);
    if (c < 0.f) w = w - n * (2.0f * c);
  }
  q = gtab_pdf(e, n, w);
  return w;
}

// ------------------------------------------------------------ BVH traversal
struct Hit { int tri; float t; };

__device__ __forceinline__ void load_node(const Node* nodes, int i, float4& a, float4& b, float4& c, int4& d) {
  const float4* p = reinterpret_cast<const float4*>(nodes + i);
  a = p[0]; b = p[1]; c = p[2];
  d = reinterpret_cast<const int4*>(nodes + i)[3];
}

__device__ __forceinline__ bool slab(float lox, float loy, float loz, float hix, float hiy, float hiz,
                                     f3 o, f3 inv, float tmin, float tmax, float& tn) {
  float tx0 = (lox - o.x) * inv.x, tx1 = (hix - o.x) * inv.x;
  float ty0 = (loy - o.y) * inv.y, ty1 = (hiy - o.y) * inv.y;
  float tz0 = (loz - o.z) * inv.z, tz1 = (hiz - o.z) * inv.z;
  float n = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), tmin));
  float f = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
  tn = n;
  return n <= f;
}

// Moller-Trumbore with inclusive edges; returns t or -1.
__device__ __forceinline__ float tri_t(const Tri* tris, int k, f3 o, f3 d, int& prim) {
  const float4* p = reinterpret_cast<const float4*>(tris + k);
  float4 A = p[0], B = p[1], C = p[2];
  prim = __float_as_int(A.w);
  LT_COUNT(3, 1);
  f3 p0 = {A.x, A.y, A.z}, e1 = {B.x, B.y, B.z}, e2 = {C.x, C.y, C.z};
  f3 pv = cross(d, e2);
  float det = dot(e1, pv);
  if (det == 0.0f) return -1.0f;
  float inv = 1.0f / det;
  f3 tv = o - p0;
  float b1 = dot(tv, pv) * inv;
  if (b1 < 0.0f || b1 > 1.0f) return -1.0f;
  f3 q = cross(tv, e1);
  float b2 = dot(d, q) * inv;
  if (b2 < 0.0f || b1 + b2 > 1.0f) return -1.0f;
  return dot(e2, q) * inv;
}

__device__ __forceinline__ f3 safe_inv(f3 d) {
  return {1.0f / d.x, 1.0f / d.y, 1.0f / d.z};
}

// ------------------------------------------------------------ heightfield
// The heightfield's triangles are not in the BVH: a ray walks the grid
// cells its (x, z) projection crosses inside the heightfield's bounding box
// (footprint x [x0, x0 + (G-1) dx], z likewise, y between the least and the
// greatest height), in order along the ray, and tests the two triangles of
// each cell (slots n_static + 2 cell + half).  A hit inside a cell lies in
// that cell's stretch of the ray, so the walk stops at the first cell that
// starts beyond the best hit; cells that start exactly at it are still
// tested, for the tie rule.  The grid's heights (G^2 floats) and triangles
// stay cache-resident where a BVH over them (16 MB of nodes at G = 256)
// did not, and a ray crosses a few cells where it visited ~15 BVH levels.
// Returns false when the ray misses the box; else the clipped interval.
__device__ __forceinline__ bool hf_span(const DevScene& sc, f3 o, f3 inv, float tmin, float tmax, float& t0,
                                        float& t1) {
  const float ext = (float)(sc.hf_G - 1) * sc.hf_dx;
  const float xl = sc.hf_x0, xh = sc.hf_x0 + ext, zl = sc.hf_z0, zh = sc.hf_z0 + ext;
  const float yl = sc.hf_base + sc.hf_hb[0], yh = sc.hf_base + sc.hf_hb[1];
  const float px = 1e-5f + 1e-6f * fmaxf(fabsf(xl), fabsf(xh)), pz = 1e-5f + 1e-6f * fmaxf(fabsf(zl), fabsf(zh));
  const float py = 1e-5f + 1e-6f * fmaxf(fabsf(yl), fabsf(yh));
  float tn;
  if (!slab(xl - px, yl - py, zl - pz, xh + px, yh + py, zh + pz, o, inv, tmin, tmax, tn)) return false;
  float tx0 = (xl - px - o.x) * inv.x, tx1 = (xh + px - o.x) * inv.x;
  float ty0 = (yl - py - o.y) * inv.y, ty1 = (yh + py - o.y) * inv.y;
  float tz0 = (zl - pz - o.z) * inv.z, tz1 = (zh + pz - o.z) * inv.z;
  t0 = tn;
  t1 = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax));
  return true;
}

// Walks the cells of the span; visit(slot0 of the cell) returns true to stop
// (any-hit), and `limit` is re-read after every cell (closest hit).
template <typename Visit>
__device__ __forceinline__ void hf_walk(const DevScene& sc, f3 o, f3 d, f3 inv, float t0, float t1,
                                        const float& limit, Visit visit) {
  const int G = sc.hf_G, last = G - 2;
  const float dx = sc.hf_dx, idx = 1.0f / dx;
  const float xs = o.x + d.x * t0, zs = o.z + d.z * t0;
  int ci = min(max((int)floorf((xs - sc.hf_x0) * idx), 0), last);
  int cj = min(max((int)floorf((zs - sc.hf_z0) * idx), 0), last);
  const int sx = d.x > 0.0f ? 1 : -1, sz = d.z > 0.0f ? 1 : -1;
  for (int it = 0; it < 2 * G; ++it) {
    if (visit(sc.n_static + 2 * (cj * (G - 1) + ci))) return;
    // where the ray leaves this cell in x and in z (from the cell index, no drift)
    const float tX = d.x != 0.0f ? (sc.hf_x0 + (float)(ci + (sx > 0)) * dx - o.x) * inv.x : 3.0e38f;
    const float tZ = d.z != 0.0f ? (sc.hf_z0 + (float)(cj + (sz > 0)) * dx - o.z) * inv.z : 3.0e38f;
    const float tn = fminf(tX, tZ);
    if (!(tn <= fminf(limit, t1))) return;
    if (tX < tZ) { ci += sx; if (ci < 0 || ci > last) return; }
    else { cj += sz; if (cj < 0 || cj > last) return; }
  }
}

// The static triangles' part: the BVH.
__device__ __forceinline__ void bvh_closest(const DevScene& sc, f3 o, f3 d, float tmin, Hit& h, int& best_prim,
                                            int* stk, int ss) {
  f3 inv = safe_inv(d);
  int sp = 0, node = 0;
  while (true) {
    float4 a, b, c; int4 e4;
    load_node(sc.nodes, node, a, b, c, e4);
    // plain scalars: a select over the vector's fields would be lowered
    // to an indexed private-memory access
    const struct { int x, y, z, w; } e = {e4.x, e4.y, e4.z, e4.w};
    LT_COUNT(2, 1);
    float tn0, tn1;
    bool h0 = e.x >= 0 && slab(a.x, a.y, a.z, a.w, b.x, b.y, o, inv, tmin, h.t, tn0);
    bool h1 = e.y >= 0 && slab(b.z, b.w, c.x, c.y, c.z, c.w, o, inv, tmin, h.t, tn1);
    if (h0 && e.z > 0) {
      for (int k = e.x; k < e.x + e.z; ++k) {
        int prim; float t = tri_t(sc.tris, k, o, d, prim);
        if (t > tmin && (t < h.t || (t == h.t && prim < best_prim))) { h.t = t; h.tri = k; best_prim = prim; }
      }
      h0 = false;
    }
    if (h1 && e.w > 0) {
      for (int k = e.y; k < e.y + e.w; ++k) {
        int prim; float t = tri_t(sc.tris, k, o, d, prim);
        if (t > tmin && (t < h.t || (t == h.t && prim < best_prim))) { h.t = t; h.tri = k; best_prim = prim; }
      }
      h1 = false;
    }
    if (h0 && h1) {
      int nearc = tn0 <= tn1 ? e.x : e.y, farc = tn0 <= tn1 ? e.y : e.x;
      stk[sp * ss] = farc; ++sp;
      node = nearc;
    } else if (h0) {
      node = e.x;
    } else if (h1) {
      node = e.y;
    } else {
      if (sp == 0) break;
      --sp; node = stk[sp * ss];
    }
  }
}


// Closest hit with t in (tmin, tmax): smallest t, ties to the lower
// primitive id.  `stk` is this lane's LDS stack slice (stride `ss`).
// HF = false: a kernel instantiated for scenes without a heightfield (the
// grid walk's registers then cost it nothing).
template <bool HF = true>
__device__ __forceinline__ Hit closest_hit(const DevScene& sc, f3 o, f3 d, float tmin, float tmax,
                                           int* stk, int ss) {
  LT_COUNT(0, 1);
  Hit h{-1, tmax};
  int best_prim = 0x7fffffff;
  if (sc.n_nodes > 0) bvh_closest(sc, o, d, tmin, h, best_prim, stk, ss);
  if (HF && sc.hf_G >= 2) {
    const f3 inv = safe_inv(d);
    float t0, t1;
    if (hf_span(sc, o, inv, tmin, h.t, t0, t1))
      hf_walk(sc, o, d, inv, t0, t1, h.t, [&](int s0) {
        for (int k = s0; k < s0 + 2; ++k) {
          int prim; float t = tri_t(sc.tris, k, o, d, prim);
          if (t > tmin && (t < h.t || (t == h.t && prim < best_prim))) { h.t = t; h.tri = k; best_prim = prim; }
        }
        return false;
      });
  }
  return h;
}

// Any static triangle with t in (tmin, tmax): the BVH.
__device__ __forceinline__ bool bvh_any(const DevScene& sc, f3 o, f3 d, float tmin, float tmax, int* stk, int ss) {
  f3 inv = safe_inv(d);
  int sp = 0, node = 0;
  while (true) {
    float4 a, b, c; int4 e4;
    load_node(sc.nodes, node, a, b, c, e4);
    // plain scalars: a select over the vector's fields would be lowered
    // to an indexed private-memory access
    const struct { int x, y, z, w; } e = {e4.x, e4.y, e4.z, e4.w};
    LT_COUNT(2, 1);
    float tn0, tn1;
    bool h0 = e.x >= 0 && slab(a.x, a.y, a.z, a.w, b.x, b.y, o, inv, tmin, tmax, tn0);
    bool h1 = e.y >= 0 && slab(b.z, b.w, c.x, c.y, c.z, c.w, o, inv, tmin, tmax, tn1);
    if (h0 && e.z > 0) {
      for (int k = e.x; k < e.x + e.z; ++k) {
        int prim; float t = tri_t(sc.tris, k, o, d, prim);
        if (t > tmin && t < tmax) return true;
      }
      h0 = false;
    }
    if (h1 && e.w > 0) {
      for (int k = e.y; k < e.y + e.w; ++k) {
        int prim; float t = tri_t(sc.tris, k, o, d, prim);
        if (t > tmin && t < tmax) return true;
      }
      h1 = false;
    }
    if (h0 && h1) {
      stk[sp * ss] = e.y; ++sp;
      node = e.x;
    } else if (h0) {
      node = e.x;
    } else if (h1) {
      node = e.y;
    } else {
      if (sp == 0) break;
      --sp; node = stk[sp * ss];
    }
  }
  return false;
}

// Any hit with t in (tmin, tmax).
template <bool HF = true>
__device__ __forceinline__ bool any_hit(const DevScene& sc, f3 o, f3 d, float tmin, float tmax,
                                        int* stk, int ss) {
  LT_COUNT(1, 1);
  if (sc.n_nodes > 0 && bvh_any(sc, o, d, tmin, tmax, stk, ss)) return true;
  if (!HF || sc.hf_G < 2) return false;
  const f3 inv = safe_inv(d);
  float t0, t1;
  if (!hf_span(sc, o, inv, tmin, tmax, t0, t1)) return false;
  bool hit = false;
  hf_walk(sc, o, d, inv, t0, t1, tmax, [&](int s0) {
    for (int q = s0; q < s0 + 2; ++q) {
      int prim; float t = tri_t(sc.tris, q, o, d, prim);
      if (t > tmin && t < tmax) { hit = true; break; }
    }
    return hit;
  });
  return hit;
}

// ------------------------------------------------------------ path pieces
struct Ray { f3 x, w, offn; bool off; };

// Vertex 0: position on the emitter and emitted direction; returns the
// initial throughput factor (beta_0 = L_e * factor).
__device__ __forceinline__ float emit(const DevScene& sc, uint64_t seed, uint32_t path, Ray& r) {
  LT_COUNT(7, 1);
  u4f u = rng4(seed, path, 0u, 0u);
  if (sc.em_type == 2) {  // directional: a collimated beam along the quad's normal
    f3 o = ld3(sc.em_o), e1 = ld3(sc.em_e1), e2 = ld3(sc.em_e2), ne = ld3(sc.em_n);
    r.x = o + e1 * u.u0 + e2 * u.u1;
    r.w = ne;
    r.offn = ne; r.off = true;
    return sc.em_area;
  }
  if (sc.em_type == 0) {
    f3 o = ld3(sc.em_o), e1 = ld3(sc.em_e1), e2 = ld3(sc.em_e2), ne = ld3(sc.em_n);
    r.x = o + e1 * u.u0 + e2 * u.u1;
    r.w = cosine_dir(ne, u.u2, u.u3);
    r.offn = ne; r.off = true;
    return sc.em_area * 3.14159265358979323846f;
  }
  r.x = ld3(sc.em_o);
  float z = 1.0f - 2.0f * u.u2;
  float rr = sqrtf(fmaxf(0.0f, 1.0f - z * z));
  r.w = {rr * cospif(2.0f * u.u3), rr * sinpif(2.0f * u.u3), z};
  r.offn = {0.f, 0.f, 0.f}; r.off = false;
  return 4.0f * 3.14159265358979323846f;
}

__device__ __forceinline__ f3 ray_origin(const Ray& r) {
  if (!r.off) return r.x;
  return r.x + r.offn * (dot(r.w, r.offn) >= 0.0f ? kEps : -kEps);
}

// Hit point recomputed from the true origin on the hit triangle's plane,
// with barycentrics and the unit geometric normal.
struct Surf { f3 x, ng; float b1, b2; int prim; };

__device__ __forceinline__ Surf surface(const DevScene& sc, int k, const Ray& r) {
  const float4* p = reinterpret_cast<const float4*>(sc.tris + k);
  float4 A = p[0], B = p[1], C = p[2];
  f3 p0 = {A.x, A.y, A.z}, e1 = {B.x, B.y, B.z}, e2 = {C.x, C.y, C.z};
  f3 N = cross(e1, e2);
  float t = dot(p0 - r.x, N) / dot(r.w, N);
  Surf s;
  s.x = r.x + r.w * t;
  float nn = dot(N, N);
  f3 dx = s.x - p0;
  s.b1 = dot(cross(dx, e2), N) / nn;
  s.b2 = dot(cross(e1, dx), N) / nn;
  s.ng = N * (1.0f / sqrtf(nn));
  s.prim = __float_as_int(A.w);
  return s;
}

__device__ __forceinline__ int texel_of(const DevScene& sc, const Surf& s, int tex) {
  const int R = sc.tex_res;
  float uvx = 0.f, uvy = 0.f;
  if (s.prim < sc.n_static) {
    const float* uv = sc.prim_uv + (size_t)s.prim * 6;
    float c0 = 1.0f - s.b1 - s.b2;
    uvx = c0 * uv[0] + s.b1 * uv[2] + s.b2 * uv[4];
    uvy = c0 * uv[1] + s.b1 * uv[3] + s.b2 * uv[5];
  }
  int tx = (int)floorf(uvx * R), ty = (int)floorf(uvy * R);
  tx = min(max(tx, 0), R - 1);
  ty = min(max(ty, 0), R - 1);
  return (tex * R + ty) * R + tx;
}

// Sensor connection geometry at a Lambertian vertex (Eq. 1 term i):
// returns true with film position u and factor g (C = beta * rho * g) when
// the camera sees x from the side the light arrived on, unoccluded.
// visible = true: the caller already knows the shadow ray is unoccluded
// (a replay of a connection found valid earlier); the test is skipped.
// A conductor vertex passes its arrival-side shading normal na and
// roughness a: the camera must lie on na's side too, and g carries the
// microfacet factor instead of the Lambertian cos / pi.
template <bool HF = true>
__device__ __forceinline__ bool connect(const DevScene& sc, const Surf& s, f3 w_in, float Kfilm,
                                        float& ux, float& uy, float& g, int* stk, int ss,
                                        bool visible = false, const f3* na = nullptr, float a = 0.f) {
  f3 cpos = ld3(sc.cpos);
  f3 dv = s.x - cpos;
  float zc = dot(dv, ld3(sc.cf));
  if (!(zc > 0.0f)) return false;
  float qx = dot(dv, ld3(sc.cr)) / zc, qy = dot(dv, ld3(sc.cu)) / zc;
  ux = 0.5f * sc.W * (1.0f + qx / (sc.aspect * sc.tan_half));
  uy = 0.5f * sc.H * (1.0f - qy / sc.tan_half);
  if (!(ux >= 0.0f && ux < (float)sc.W && uy >= 0.0f && uy < (float)sc.H)) return false;
  float dist2 = dot(dv, dv);
  float dist = sqrtf(dist2);
  f3 wc = dv * (-1.0f / dist);
  float cg = dot(s.ng, wc);
  float cos_in = dot(w_in, s.ng);
  if (!(cg * (-cos_in) > 0.0f)) return false;
  if (na && !(dot(*na, wc) > 0.0f)) return false;
  f3 so = s.x + s.ng * (cg >= 0.0f ? kEps : -kEps);
  f3 sd = cpos - so;
  float sl = sqrtf(dot(sd, sd));
  sd = sd * (1.0f / sl);
  if (!visible && any_hit<HF>(sc, so, sd, kTmin, sl * (1.0f - 1e-4f), stk, ss)) return false;
  float cosc = zc / dist;
  if (na) {
    g = Kfilm * ggx_conn(w_in * -1.0f, wc, *na, a) / (cosc * cosc * cosc * dist2);
  } else {
    float cosx = fabsf(dot(s.ng, dv)) / dist;
    g = 0.31830988618379067f * Kfilm * cosx / (cosc * cosc * cosc * dist2);
  }
  return true;
}

// Tent reconstruction filter of radius one pixel: the four taps around u
// with weights F(u, p), taps outside the film dropped (weight 0).
struct Taps { int idx[4]; float w[4]; };

__device__ __forceinline__ Taps tent_taps(const DevScene& sc, float ux, float uy) {
  Taps t;
  float fx = ux - 0.5f, fy = uy - 0.5f;
  int px0 = (int)floorf(fx), py0 = (int)floorf(fy);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int px = px0 + (q & 1), py = py0 + (q >> 1);
    float wx = 1.0f - fabsf(ux - ((float)px + 0.5f));
    float wy = 1.0f - fabsf(uy - ((float)py + 0.5f));
    bool in = px >= 0 && px < sc.W && py >= 0 && py < sc.H;
    t.idx[q] = in ? (py * sc.W + px) * 3 : -1;
    t.w[q] = in ? wx * wy : 0.0f;
  }
  return t;
}

__device__ __forceinline__ void splat(const DevScene& sc, float* image, float ux, float uy, f3 C) {
  LT_COUNT(4, 1);
  Taps t = tent_taps(sc, ux, uy);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (t.idx[q] < 0) continue;
    float* p = image + t.idx[q];
    atomicAdd(p + 0, t.w[q] * C.x);
    atomicAdd(p + 1, t.w[q] * C.y);
    atomicAdd(p + 2, t.w[q] * C.z);
  }
}

// Wave-cooperative tent splat.  Float atomics to device memory are
// executed past the L2, so their cost scales with the number of distinct
// cache lines an instruction touches.  The lanes holding a splat are
// processed five at a time: lane l adds value l%12 (2 rows x 2 taps x RGB)
// of splat l/12, so each atomic instruction covers five splats' contiguous
// tap rows instead of 64 unrelated addresses.  Must be called by all lanes
// of the wave (has = false for lanes without a splat).
__device__ __forceinline__ void splat_wave(const DevScene& sc, float* image, bool has, float ux, float uy, f3 C) {
  uint64_t m = __ballot(has);
  if (m == 0ull) return;
  LT_COUNT(4, has ? 1 : 0);
  int px0 = (int)floorf(ux - 0.5f), py0 = (int)floorf(uy - 0.5f);
  const int lane = __lane_id();
  const int slot = lane / 12, v = lane - slot * 12;
  const int row = v / 6, k = v - row * 6, tx = k / 3, ch = k - tx * 3;
  while (m) {
    // the next five pending splats in lane order, found on the wave-uniform
    // mask (-1 past the last); lane slot s takes the s-th
    uint64_t r = m;
    int b[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      b[i] = r ? __ffsll((unsigned long long)r) - 1 : -1;
      r &= r - 1ull;
    }
    const int pick = slot == 0 ? b[0] : slot == 1 ? b[1] : slot == 2 ? b[2] : slot == 3 ? b[3] : slot == 4 ? b[4] : -1;
    const bool act = pick >= 0;
    const int src = act ? pick : 0;
    int spx = __shfl(px0, src), spy = __shfl(py0, src);
    float sux = __shfl(ux, src), suy = __shfl(uy, src);
    float c0 = __shfl(C.x, src), c1 = __shfl(C.y, src), c2 = __shfl(C.z, src);
    int px = spx + tx, py = spy + row;
    if (act && px >= 0 && px < sc.W && py >= 0 && py < sc.H) {
      float wx = 1.0f - fabsf(sux - ((float)px + 0.5f));
      float wy = 1.0f - fabsf(suy - ((float)py + 0.5f));
      float c = ch == 0 ? c0 : (ch == 1 ? c1 : c2);
      atomicAdd(image + (py * sc.W + px) * 3 + ch, wx * wy * c);
    }
    m = r;
  }
}

// Lane position of the s-th (from 0) set bit of m, which has more than s set
// bits: the largest p with fewer than s + 1 set bits below it, by binary
// lifting on popcounts (six steps, the same for every lane).
__device__ __forceinline__ int nth_set_bit(uint64_t m, int s) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w > 0; w >>= 1)
    if (__popcll(m & ((1ull << (pos + w)) - 1ull)) <= s) pos += w;
  return pos;
}

// Wave-cooperative add of RGB triplets: every lane with `has` adds v to
// dst[3*idx .. 3*idx+2]; 21 triplets per atomic instruction, zero values
// skipped.  Must be called by all lanes of the wave.
__device__ __forceinline__ void scatter3_wave(float* dst, bool has, int idx, f3 v) {
  uint64_t m = __ballot(has);
  if (m == 0ull) return;
  LT_COUNT(6, has ? 3 : 0);
  const int lane = __lane_id();
  // Same-address atomics serialize: when many lanes target the index of
  // the first pending lane (a small or constant texture), sum them across
  // the wave first and let one lane commit.
  for (int rep = 0; rep < 2 && m; ++rep) {
    int lead = __ffsll((unsigned long long)m) - 1;
    int li = __shfl(idx, lead);
    bool mine = has && ((m >> lane) & 1ull) && idx == li;
    uint64_t same = __ballot(mine);
    if (__popcll(same) < 8) break;
    float s0 = mine ? v.x : 0.f, s1 = mine ? v.y : 0.f, s2 = mine ? v.z : 0.f;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_xor(s0, o); s1 += __shfl_xor(s1, o); s2 += __shfl_xor(s2, o);
    }
    if (lane == lead) {
      if (s0 != 0.f) atomicAdd(dst + (size_t)li * 3 + 0, s0);
      if (s1 != 0.f) atomicAdd(dst + (size_t)li * 3 + 1, s1);
      if (s2 != 0.f) atomicAdd(dst + (size_t)li * 3 + 2, s2);
    }
    m &= ~same;
  }
  if (m == 0ull) return;
  has = has && ((m >> lane) & 1ull);
  const int slot = lane / 3, ch = lane - slot * 3;
  while (m) {
    // lane slot s takes the s-th pending triplet
    const bool act = slot < 21 && slot < __popcll(m);
    const int src = act ? nth_set_bit(m, slot) : 0;
    int sidx = __shfl(idx, src);
    float c0 = __shfl(v.x, src), c1 = __shfl(v.y, src), c2 = __shfl(v.z, src);
    float c = ch == 0 ? c0 : (ch == 1 ? c1 : c2);
    if (act && c != 0.0f) atomicAdd(dst + (size_t)sidx * 3 + ch, c);
    for (int i = 0; i < 21 && m; ++i) m &= m - 1ull;
  }
}

// Filter-matched adjoint read: sum over taps of F(u, p) dI[p].
__device__ __forceinline__ f3 gather(const DevScene& sc, const float* dI, float ux, float uy) {
  LT_COUNT(5, 1);
  Taps t = tent_taps(sc, ux, uy);
  f3 a = {0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (t.idx[q] < 0) continue;
    const float* p = dI + t.idx[q];
    a = a + mk(p[0], p[1], p[2]) * t.w[q];
  }
  return a;
}

// Dielectric lobe choice and direction (weight 1): unpolarized Fresnel with
// the shading normal ns (unit, same side as ng); the path ends when
// cos_i <= 0 against the shading normal or the new direction falls on the
// wrong side of the geometric normal.
// Return value: 0 ok, 7 cos_i <= 0, 8 wrong side.
__device__ __forceinline__ int dielectric(f3 w_in, f3 ng, f3 ns, float ior, float u_lobe, f3& wo,
                                          bool& reflect, float& cos_t) {
  float cos_g = dot(w_in, ng);
  bool entering = cos_g < 0.0f;
  float eta = entering ? 1.0f / ior : ior;
  f3 n = entering ? ns : ns * -1.0f;
  float cosi = -dot(w_in, n);
  if (!(cosi > 0.0f)) { reflect = false; return 7; }
  float sin2t = eta * eta * (1.0f - cosi * cosi);
  float F, cost = 0.0f;
  if (sin2t >= 1.0f) F = 1.0f;
  else {
    cost = sqrtf(1.0f - sin2t);
    float ei = entering ? 1.0f : ior, et = entering ? ior : 1.0f;
    float rs = (ei * cosi - et * cost) / (ei * cosi + et * cost);
    float rp = (et * cosi - ei * cost) / (et * cosi + ei * cost);
    F = 0.5f * (rs * rs + rp * rp);
  }
  reflect = u_lobe < F;
  cos_t = reflect ? 1.0f : cost;
  if (reflect) wo = w_in + n * (2.0f * cosi);
  else wo = w_in * eta + n * (eta * cosi - cost);
  float side_in = -cos_g, s_out = dot(wo, ng);
  if (reflect ? (s_out * side_in <= 0.0f) : (s_out * side_in >= 0.0f)) return 8;
  return 0;
}

// Heightfield shading normal: barycentric blend of the corners'
// central-difference slopes, n = normalize(-Sx, 1, -Sz).
__device__ __forceinline__ float hget(const float* h, int G, int i, int j) { return h ? h[j * G + i] : 0.0f; }

__device__ __forceinline__ void hf_corner(int G, int local, int k, int& gi, int& gj) {
  int cell = local >> 1, half = local & 1;
  int ci = cell % (G - 1), cj = cell / (G - 1);
  // half 0: (A, C, B); half 1: (A, D, C)
  int oi = half == 0 ? (k == 0 ? 0 : 1) : (k == 2 ? 1 : 0);
  int oj = half == 0 ? (k == 1 ? 1 : 0) : (k == 0 ? 0 : 1);
  gi = ci + oi; gj = cj + oj;
}

__device__ __forceinline__ void hf_slope(const float* h, int G, float dx, int i, int j, float& sx, float& sz) {
  int a = max(i - 1, 0), b = min(i + 1, G - 1);
  sx = (hget(h, G, b, j) - hget(h, G, a, j)) / ((float)(b - a) * dx);
  int c = max(j - 1, 0), d = min(j + 1, G - 1);
  sz = (hget(h, G, i, d) - hget(h, G, i, c)) / ((float)(d - c) * dx);
}

// Shading slopes at grid vertex (i, j): the normal-map parameters (Sx, Sz)
// of a normal-mapped surface when nmap is given, else the central
// differences of the heights.
__device__ __forceinline__ void hf_slopes(const float* h, const float* nmap, int G, float dx, int i, int j, float& sx,
                                          float& sz) {
  if (nmap) {
    const float* q = nmap + 2 * (j * G + i);
    sx = q[0]; sz = q[1];
    return;
  }
  hf_slope(h, G, dx, i, j, sx, sz);
}

__device__ __forceinline__ f3 hf_shading_normal(const DevScene& sc, const float* h, const float* nmap, const Surf& s) {
  int local = s.prim - sc.n_static;
  float Sx = 0.f, Sz = 0.f;
  float wts[3] = {1.0f - s.b1 - s.b2, s.b1, s.b2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int gi, gj; hf_corner(sc.hf_G, local, k, gi, gj);
    float sx, sz; hf_slopes(h, nmap, sc.hf_G, sc.hf_dx, gi, gj, sx, sz);
    Sx += wts[k] * sx; Sz += wts[k] * sz;
  }
  return normalize(mk(-Sx, 1.0f, -Sz));
}

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint64_t lanemask_lt() {
  return (1ull << __lane_id()) - 1ull;
}

// XCD (accelerator complex die) of the executing workgroup: hardware
// register XCC_ID, bits 3:0.  A workgroup stays on its XCD.
__device__ __forceinline__ int xcd_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 7; }

// A wave's place in the work distribution: the counter block of the pass,
// the residue class it draws from and how many classes it has found used up.
struct WorkQ { unsigned int* base; int cls; int tried; };
__device__ __forceinline__ WorkQ work_begin(unsigned int* base) { return {base, xcd_id(), 0}; }

// Wave-aggregated work fetch: every lane with `need` set gets the next
// unused index of `counter` (one atomic per wave).
__device__ __forceinline__ uint32_t fetch_paths(unsigned int* counter, bool need) {
  uint64_t m = __ballot(need);
  unsigned int base = 0;
  int leader = __ffsll((unsigned long long)m) - 1;
  if (m && __lane_id() == leader) base = atomicAdd(counter, (unsigned int)__popcll(m));
  base = __shfl(base, leader < 0 ? 0 : leader);
  return base + (uint32_t)__popcll(m & lanemask_lt());
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

}  // namespace lt
