// gfx950 kernels of the light tracer and its three reverse modes.
//
// Every pass is a persistent kernel: each wave keeps all 64 lanes busy by
// fetching new path indices (one atomic per wave) as soon as lanes finish
// their path, so paths of uneven length do not idle the SIMD.  All path
// state lives in registers; the BVH traversal stack lives in LDS.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#include "lt_device.h"
#include "lt_launch.h"

namespace lt {

// The instrumented build (event counters on) gives its kernels their own
// symbol names so that profiles keep the two builds apart.
#ifdef LT_COUNTERS
inline namespace counted {
#endif

// One vertex of a light path: closest hit, material dispatch, sensor
// connection geometry and the sampling of the next direction.
struct Event {
  int prim;        // hit primitive, -1 on a miss
  int kind;        // 0 path ended at this hit (miss/absorber), 1 Lambertian or rough
                   // conductor (a texel, a connection, a scatter linear in rho), 2 dielectric
  bool cond;       // kind 1 on a rough conductor
  int texel;       // Lambertian texel
  f3 rho;          // Lambertian albedo
  bool valid;      // sensor connection exists
  float ux, uy, g; // film position and connection factor (C = beta rho g)
  float cos_in;
  int lobe, fail;  // dielectric: lobe 2 reflect / 4 refract, fail 7/8; conductor: fail 9
                   // (arrived behind its shading normal), 7/8 (no reflection)
  bool cont;       // the path continues with the updated ray
  float u_res;     // reservoir uniform of this vertex
  int slot;        // hit triangle in BVH order
  f3 x;            // hit point
  float gw, gq;    // Lambertian scatter weight over rho (cos / (pi q) when guided, else 1)
                   // and the guided density q (0: cosine sampling)
  int gcomp;       // guided component (0 cosine, k + 1 lobe k)
  bool illc;       // ill-conditioned vertex for attached derivatives (grazing hit,
                   // refraction near the critical angle, short segment, or a
                   // connection next to a tent-filter kink)
};

__device__ __forceinline__ bool near_kink(float u) {
  float d = u - 0.5f;
  return fabsf(d - rintf(d)) < 1e-3f;
}

// cmode: 0 no sensor connection, 1 full connection test (with shadow
// ray), 2 connection geometry only (known visible from an earlier replay).
template <bool HF = true>
__device__ __forceinline__ Event bounce(const PassArgs& A, uint32_t path, int j, Ray& r, int cmode,
                                        int* stk, int ss) {
  const DevScene& sc = A.sc;
  Event ev;
  ev.prim = -1; ev.kind = 0; ev.cond = false; ev.texel = -1; ev.rho = {0.f, 0.f, 0.f}; ev.valid = false;
  ev.ux = ev.uy = ev.g = 0.f; ev.lobe = 0; ev.fail = 0; ev.cont = false; ev.u_res = 1.0f; ev.cos_in = 0.f;
  ev.slot = -1; ev.x = {0.f, 0.f, 0.f}; ev.illc = false; ev.gw = 1.0f; ev.gq = 0.f; ev.gcomp = 0;
  Hit h = closest_hit<HF>(sc, ray_origin(r), r.w, kTmin, 3.0e38f, stk, ss);
  if (h.tri < 0) return ev;
  Surf s = surface(sc, h.tri, r);
  ev.prim = s.prim;
  ev.slot = h.tri;
  ev.x = s.x;
  int mat = sc.prim_mat[s.prim];
  int mt = sc.mat_type[mat];
  if (mt == 0) return ev;
  ev.cos_in = dot(r.w, s.ng);
  // grazing hit (hit-point derivatives ~ 1/cos) or a short segment (the
  // segment direction carries position rounding amplified by 1/length)
  f3 seg = s.x - r.x;
  ev.illc = fabsf(ev.cos_in) < 0.02f || dot(seg, seg) < 4e-4f;
  u4f u = (mt != 2 || j < A.D) ? rng4(A.seed, path, (uint32_t)j, 0u) : u4f{0.f, 0.f, 0.f, 1.f};
  ev.u_res = u.u3;
  if (mt == 1 || mt == 3) {
    ev.kind = 1;
    ev.cond = mt == 3;
    ev.texel = texel_of(sc, s, sc.mat_tex[mat]);
    ev.rho = ld3(A.albedo + (size_t)ev.texel * 3);
    f3 nc = s.ng;  // conductor: arrival-side shading normal
    float rough = 0.f;
    if (ev.cond) {
      rough = sc.mat_ior[mat];
      f3 ns = s.prim >= sc.n_static ? hf_shading_normal(sc, A.heights, A.nmap, s) : s.ng;
      nc = ev.cos_in < 0.0f ? ns : ns * -1.0f;
      if (!(dot(r.w, nc) < 0.0f)) { ev.fail = 9; return ev; }
    }
    if (cmode)
      ev.valid = connect<HF>(sc, s, r.w, A.Kfilm, ev.ux, ev.uy, ev.g, stk, ss, cmode == 2, ev.cond ? &nc : nullptr, rough);
    // the tent filter has kinks where u - 1/2 is an integer: within 1e-3 px
    // of one the splat-position derivative is one-sided (rounding picks the side)
    if (ev.valid && (near_kink(ev.ux) || near_kink(ev.uy))) ev.illc = true;
    if (j < A.D && ev.cond) {
      f3 wo;
      float wgt;
      int code = conductor_scatter(r.w * -1.0f, nc, s.ng, ev.cos_in < 0.0f ? 1.0f : -1.0f, rough, u.u0, u.u1, wo, wgt);
      if (code) { ev.fail = code; return ev; }
      ev.gw = wgt;
      r.w = wo; r.x = s.x; r.offn = s.ng; r.off = true;
      ev.cont = true;
      return ev;
    }
    if (j < A.D) {
      f3 na = ev.cos_in < 0.0f ? s.ng : s.ng * -1.0f;
      const float4* ge = A.gtab ? A.gtab + (size_t)(2 * ev.texel + (ev.cos_in < 0.0f ? 0 : 1)) * kGTabF4 : nullptr;
      if (ge && ge[1].w >= 0.f) {
        // guided scatter (component by u2, direction by u0, u1), weight
        // f cos / q = rho cos / (pi q) with q held fixed
        float q;
        int comp;
        f3 w = gtab_sample(ge, na, u.u2, u.u0, u.u1, q, comp);
        ev.gcomp = comp;
        float c = dot(w, na);
        if (!(q > 0.f && c > 0.f)) return ev;
        ev.gw = c / (3.14159265358979323846f * q);
        ev.gq = q;
        r.w = w;
      } else {
        r.w = cosine_dir(na, u.u0, u.u1);
      }
      r.x = s.x; r.offn = s.ng; r.off = true;
      ev.cont = true;
    }
    return ev;
  }
  ev.kind = 2;
  if (j >= A.D) return ev;
  f3 ns = s.ng;
  if (s.prim >= sc.n_static) ns = hf_shading_normal(sc, A.heights, A.nmap, s);
  f3 wo; bool refl;
  float cos_t = 1.f;
  int code = dielectric(r.w, s.ng, ns, sc.mat_ior[mat], u.u2, wo, refl, cos_t);
  if (code == 7) { ev.fail = 7; return ev; }
  ev.lobe = refl ? 2 : 4;
  // refraction near the critical angle: d(cos_t) ~ 1/cos_t amplifies FP32
  // rounding of the primal direction by ~1/cos_t^2 in the derivatives
  if (cos_t < 0.1f) ev.illc = true;
  if (code == 8) { ev.fail = 8; return ev; }
  r.w = wo; r.x = s.x; r.offn = s.ng; r.off = true;
  ev.cont = true;
  return ev;
}

__device__ __forceinline__ uint32_t sig_event(uint32_t h, const Event& ev) {
  if (ev.prim < 0) return fnv1a(h, 0u);
  h = fnv1a(h, (uint32_t)ev.prim + 1u);
  if (ev.kind == 1) {
    h = fnv1a(h, (uint32_t)ev.texel + 1u);
    if (ev.fail == 9) return fnv1a(h, 9u);
    h = fnv1a(h, ev.valid ? 1u : 0u);
    if (ev.fail) h = fnv1a(h, (uint32_t)ev.fail);
  } else if (ev.kind == 2) {
    if (ev.fail == 7) return fnv1a(h, 7u);
    if (ev.lobe) h = fnv1a(h, (uint32_t)ev.lobe);
    if (ev.fail == 8) h = fnv1a(h, 8u);
  }
  return h;
}

// Work distribution.  Path indices are dealt out by eight counters,
// counter c handing out p = 8k + c (k = 0, 1, ...), each on a cache line of
// its own: with one counter for all the waves of the chip, its line was the
// busiest address of a pass and its returning atomics serialised (measured:
// the box forward 5.8 -> 4.3 ms, the fused LRB-3 backward 8.4 -> 6.8 ms).
// A wave starts on the counter of its XCD and, once that class is used up,
// moves to the next; having found all eight used up, it is done.  Every
// index below n_paths is handed out exactly once whatever the XCD reads.
// Paths that `accept` rejects (default: the path mask) get their per-path
// outputs cleared by `on_skip`.
// The same over any eight classes of work: class c holds limit(c) items,
// the k-th of them being index(c, k).
template <typename Limit, typename Index, typename Skip, typename Accept>
__device__ __forceinline__ void refill_classes(WorkQ& q, bool& alive, bool& exhausted, uint32_t& item, Limit limit,
                                               Index index, Skip on_skip, Accept accept) {
  while (true) {
    bool need = !alive && !exhausted;
    if (__ballot(need) == 0ull) break;
    if (q.tried == kWorkClasses) {  // every class used up
      if (need) exhausted = true;
      break;
    }
    const uint32_t k = fetch_paths(q.base + q.cls * kCtrStride, need);
    const bool over = need && k >= limit(q.cls);
    const uint32_t p = index(q.cls, k);
    if (__ballot(over) != 0ull) {  // this class is used up: the next one
      q.cls = (q.cls + 1) & (kWorkClasses - 1);
      ++q.tried;
    }
    if (need && !over) {
      if (!accept(p)) on_skip(p);
      else { alive = true; item = p; }
    }
  }
}
// paths: class c holds p = 8k + c below n_paths
template <typename Skip, typename Accept>
__device__ __forceinline__ void refill(const PassArgs& A, WorkQ& q, bool& alive, bool& exhausted, uint32_t& path,
                                       Skip on_skip, Accept accept) {
  const uint32_t N = (uint32_t)A.n_paths;
  refill_classes(
      q, alive, exhausted, path,
      [&](int c) { return N > (uint32_t)c ? (N - (uint32_t)c + (uint32_t)kWorkClasses - 1u) / (uint32_t)kWorkClasses : 0u; },
      [&](int c, uint32_t k) { return k * (uint32_t)kWorkClasses + (uint32_t)c; }, on_skip, accept);
}
template <typename Skip>
__device__ __forceinline__ void refill(const PassArgs& A, WorkQ& q, bool& alive, bool& exhausted, uint32_t& path,
                                       Skip on_skip) {
  refill(A, q, alive, exhausted, path, on_skip, [&](uint32_t p) { return !(A.mask && A.mask[p] == 0); });
}
// LRB-3 pass 3: the entries pass 2 appended, region by region
__device__ __forceinline__ void refill_hand(const PassArgs& A, WorkQ& q, bool& alive, bool& exhausted,
                                            uint32_t& item) {
  refill_classes(
      q, alive, exhausted, item, [&](int c) { return A.hand_app[c * kCtrStride]; },
      [&](int c, uint32_t k) { return (uint32_t)c * A.hand_region + k; }, [&](uint32_t) {},
      [&](uint32_t) { return true; });
}

// Pass 2's append of one entry per path that has one (`put`): grouped by the
// path's class, one atomic per class present in the wave; returns the
// entry's index (valid where put).  Every lane of the wave calls it.
__device__ __forceinline__ uint32_t hand_append(const PassArgs& A, bool put, uint32_t path) {
  const int c = (int)(path & (uint32_t)(kWorkClasses - 1));
  uint32_t slot = 0;
  bool todo = put;
  while (true) {
    const uint64_t m = __ballot(todo);
    if (m == 0ull) break;
    const int cl = __shfl(c, __ffsll((unsigned long long)m) - 1);
    const bool mine = todo && c == cl;
    const uint32_t k = fetch_paths(A.hand_app + cl * kCtrStride, mine);
    if (mine) { slot = (uint32_t)cl * A.hand_region + k; todo = false; }
  }
  return slot;
}

// Non-finite values (a division by a vanishing cosine, length or
// determinant on a degenerate path) never reach an atomic: they are dropped
// and counted in stats[1].
__device__ __forceinline__ void count_nonfinite(const PassArgs& A) {
  if (A.stats) atomicAdd(A.stats + 1, 1ull);
}
__device__ __forceinline__ void keep_finite(const PassArgs& A, bool& has, f3 v) {
  if (has && !(isfinite(v.x) && isfinite(v.y) && isfinite(v.z))) { has = false; count_nonfinite(A); }
}
// Textured-emitter gradients.  Every path adds to the texel it was emitted
// from, so a small texture takes all of them on a few cache lines, where
// the atomics serialize.  With A.legrad_lds each workgroup pre-reduces them
// in an LDS copy of the texture (`le`, past the albedo copy) and adds that
// to the caller's array once, at its end.  Every thread of the workgroup
// calls begin and end.
__device__ __forceinline__ float* legrad_begin(const PassArgs& A, int* lds) {
  float* le = reinterpret_cast<float*>(lds);
  if (!A.legrad_lds) return le;
  const int n = A.sc.em_tex_res * A.sc.em_tex_res * 3;
  for (int i = threadIdx.x; i < n; i += blockDim.x) le[i] = 0.f;
  __syncthreads();
  return le;
}
__device__ __forceinline__ void legrad_end(const PassArgs& A, float* le) {
  if (!A.legrad_lds) return;
  __syncthreads();
  if (!A.g_le_tex) return;
  const int n = A.sc.em_tex_res * A.sc.em_tex_res * 3;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    float v = le[i];
    if (v != 0.f) atomicAdd(A.g_le_tex + i, v);
  }
}

// emitter-gradient accumulation of one path, (a0, a1, a2) in place of zeros
// when any is non-finite: into the lane's FP64 sums (one radiance), or onto
// the path's texel of a textured emitter (texel >= 0; the workgroup's LDS
// copy `le` with A.legrad_lds)
__device__ __forceinline__ void add_le(const PassArgs& A, double& g0, double& g1, double& g2, double a0, double a1,
                                       double a2, int texel = -1, float* le = nullptr) {
  if (!(isfinite(a0) && isfinite(a1) && isfinite(a2))) { count_nonfinite(A); return; }
  if (texel >= 0) {
    if (!A.g_le_tex) return;
    if (A.legrad_lds) {
      float* d = le + 3 * texel;
      if (a0 != 0.0) atomicAdd(d + 0, (float)a0);
      if (a1 != 0.0) atomicAdd(d + 1, (float)a1);
      if (a2 != 0.0) atomicAdd(d + 2, (float)a2);
      return;
    }
    float* d = A.g_le_tex + 3 * texel;
    if (a0 != 0.0) atomicAdd(d + 0, (float)a0);
    if (a1 != 0.0) atomicAdd(d + 1, (float)a1);
    if (a2 != 0.0) atomicAdd(d + 2, (float)a2);
    return;
  }
  g0 += a0; g1 += a1; g2 += a2;
}

// Albedo gradients.  With A.agrad_lds each workgroup pre-reduces them in an
// LDS copy of the texture set and adds that to the caller's array once, at
// its end.  Without it (the set is large, or the copy would cost resident
// workgroups) they go to the caller's array through a one-entry
// write-combining cache per wave: sums for the texel most of the wave hits
// stay in registers while later scatters hit the same texel, so a constant
// or small texture takes one atomic per wave and texel change, not one per
// scatter.  Every thread of the workgroup calls begin and end, and every
// lane of a wave calls scatter.
// The LDS copy is addressed through a pointer derived only from the
// workgroup's LDS array, and the choice between it and the caller's array is
// a branch on the uniform flag, not a pointer select: each side then compiles
// to LDS or global atomics rather than flat ones.
struct AGrad {
  float* lds;
  int idx;  // cached texel (wave-uniform), -1 when empty
  float s0, s1, s2;
};
__device__ __forceinline__ AGrad agrad_begin(const PassArgs& A, int* lds) {
  AGrad g{reinterpret_cast<float*>(lds), -1, 0.f, 0.f, 0.f};
  if (!A.agrad_lds) return g;
  const int n = A.n_texels * 3;
  for (int i = threadIdx.x; i < n; i += blockDim.x) g.lds[i] = 0.f;
  __syncthreads();
  return g;
}
__device__ __forceinline__ void agrad_flush(const PassArgs& A, AGrad& g) {
  if (g.idx >= 0 && __lane_id() == 0) {
    float* d = A.g_albedo + (size_t)g.idx * 3;
    if (g.s0 != 0.f) atomicAdd(d + 0, g.s0);
    if (g.s1 != 0.f) atomicAdd(d + 1, g.s1);
    if (g.s2 != 0.f) atomicAdd(d + 2, g.s2);
  }
}
__device__ __forceinline__ void scatter_albedo(const PassArgs& A, AGrad& g, bool has, int texel, f3 v) {
  if (A.agrad_lds) {
    scatter3_wave(g.lds, has, texel, v);
    return;
  }
  uint64_t m = __ballot(has);
  if (m == 0ull) return;
  const int lane = __lane_id();
  int lead = __ffsll((unsigned long long)m) - 1;
  int li = __shfl(texel, lead);
  bool mine = has && texel == li;
  uint64_t same = __ballot(mine);
  if (li == g.idx || __popcll(same) >= 8) {
    LT_COUNT(6, mine ? 3 : 0);
    float s0 = mine ? v.x : 0.f, s1 = mine ? v.y : 0.f, s2 = mine ? v.z : 0.f;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {  // xor butterfly: every lane ends with the same sums
      s0 += __shfl_xor(s0, o); s1 += __shfl_xor(s1, o); s2 += __shfl_xor(s2, o);
    }
    if (li != g.idx) {
      agrad_flush(A, g);
      g.idx = li; g.s0 = 0.f; g.s1 = 0.f; g.s2 = 0.f;
    }
    g.s0 += s0; g.s1 += s1; g.s2 += s2;
    has = has && !mine;
    if (m == same) return;
  }
  scatter3_wave(A.g_albedo, has, texel, v);
}
__device__ __forceinline__ void agrad_end(const PassArgs& A, AGrad& g) {
  if (!A.agrad_lds) {
    agrad_flush(A, g);
    return;
  }
  __syncthreads();
  const int n = A.n_texels * 3;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    float v = g.lds[i];
    if (v != 0.f) atomicAdd(A.g_albedo + i, v);
  }
}

// The workgroup's next instance of a batch reuses the LDS past the traversal
// stacks: no wave may start on it before every wave has flushed the copies.
__device__ __forceinline__ void lds_grads_done(const PassArgs& A) {
  if (A.hgrad_lds || A.agrad_lds || A.legrad_lds) __syncthreads();
}
// LDS past the traversal stacks (stack_n entries per lane) and the albedo copy
__device__ __forceinline__ int* past_agrad(const PassArgs& A, int* lds, int stack_n) {
  return lds + stack_n * (int)blockDim.x + (A.agrad_lds ? A.n_texels * 3 : 0);
}

__device__ __forceinline__ void flush_le(const PassArgs& A, double g0, double g1, double g2) {
  g0 = wave_sum(g0); g1 = wave_sum(g1); g2 = wave_sum(g2);
  if (__lane_id() == 0 && A.g_Le_acc) {
    if (g0 != 0.0) atomicAdd(A.g_Le_acc + 0, g0);
    if (g1 != 0.0) atomicAdd(A.g_Le_acc + 1, g1);
    if (g2 != 0.0) atomicAdd(A.g_Le_acc + 2, g2);
  }
}

// Reciprocal emitter radiance, zero where a channel is zero: the emitter
// gradient of a path is its adjoint sum times this (computed once, not a
// double division per path).
struct D3R { double x, y, z; };
__device__ __forceinline__ D3R recip_le(f3 Le) {
  return {Le.x > 0.f ? 1.0 / Le.x : 0.0, Le.y > 0.f ? 1.0 / Le.y : 0.0, Le.z > 0.f ? 1.0 / Le.z : 0.0};
}

// Emitter radiance of a path.  One radiance: Le, iLe as set once per kernel,
// texel -1.  A textured emitter: the texel of the path's emission point
// (quad coordinates u0 along e1, u1 along e2, nearest texel; computed on the
// 24-bit integers of the uniforms, so exactly floor(u R)), its radiance and
// reciprocal.
__device__ __forceinline__ void path_emitter(const PassArgs& A, uint32_t path, f3& Le, D3R& iLe, int& texel) {
  const int R = A.sc.em_tex_res;
  if (R <= 0) return;
  u4f u = rng4(A.seed, path, 0u, 0u);
  const uint64_t k0 = (uint64_t)(u.u0 * 16777216.0f), k1 = (uint64_t)(u.u1 * 16777216.0f);
  const int tx = (int)((k0 * (uint64_t)R) >> 24), ty = (int)((k1 * (uint64_t)R) >> 24);
  texel = ty * R + tx;
  Le = ld3(A.Le + 3 * texel);
  iLe = recip_le(Le);
}

// Vertex 0 of a path.  With a guide the emitted direction and its density q
// come from the per-path record of the guide pass (same position draw);
// beta_1 = L_e * A cos / q, the density held fixed in every derivative.
__device__ __forceinline__ float emit_path(const PassArgs& A, uint32_t path, Ray& r) {
  float f = emit(A.sc, A.seed, path, r);
  if (A.guide_rec) {
    float4 g = A.guide_rec[path];
    r.w = mk(g.x, g.y, g.z);
    float c = fmaxf(dot(r.w, ld3(A.sc.em_n)), 0.f);
    f = g.w > 0.f ? A.sc.em_area * c / g.w : 0.f;
  }
  return f;
}

__device__ __forceinline__ float luminance(f3 c) { return 0.2126f * c.x + 0.7152f * c.y + 0.0722f * c.z; }

// ---------------------------------------------------------------- forward
// Light tracing with a connection + splat at every Lambertian vertex
// (Eq. 1-2, Eq. 20).  RESV: streams valid connections through a capacity-1
// weighted reservoir (Eq. 8) and records/splats the selection (Eq. 9).
// TAPE: writes the per-vertex naive-AD tape.  SPL: writes the buffered
// two-pass splat records (u_i, C_i of every valid connection, a per-path
// header).  GS: writes each path's diffuse-guide training sample (its first
// guided Lambertian scatter: position, arrival-side normal, direction,
// density, S = sum of lum(C_i) over the later connections, component).
// Each loop iteration advances every live lane by one vertex; the splat is
// issued cooperatively by the whole wave after the step.
template <bool TAPE, bool RESV, bool SPL = false, bool GS = false, bool HF = true>
__device__ __forceinline__ void trace_run(const PassArgs& A, int* lds) {
  int* stk = lds + threadIdx.x;
  const int ss = blockDim.x;
  const bool selected = (A.flags & 2u) != 0;
  bool alive = false, exhausted = false;
  uint32_t path = 0, sig = 0;
  int j = 0, nrec = 0;
  Ray r;
  f3 beta = {0.f, 0.f, 0.f};
  float Om = 0.f, omR = 0.f, uxR = 0.f, uyR = 0.f;
  int R = 0;
  f3 CR = {0.f, 0.f, 0.f};
  float fac = 0.f, Sl = 0.f;  // emission factor, path contribution sum_i lum(C_i)
  int klast = 0;              // SPL: last connection depth and validity bits
  uint64_t vmask = 0ull;
  f3 Le = ld3(A.Le);
  D3R iLe = {0.0, 0.0, 0.0};
  int etex = -1;
  float gs[12];  // GS: the sample being built (gs[10] accumulates S)
  bool gs_on = false;
  WorkQ wq = work_begin(A.counter);
  while (true) {
    refill(A, wq, alive, exhausted, path, [&](uint32_t p) {
      if (GS)
        for (int q = 0; q < 12; ++q) A.gsamp[(size_t)p * 12 + q] = 0.f;
      if (SPL) { SplatHdr z{}; A.spl_hdr[p] = z; }
      if (TAPE) A.tape_len[p] = 0;
      if (RESV && A.res) { ResRec z{}; A.res[p] = z; }
      if (A.sig) A.sig[p] = 0u;
      if (A.contrib) A.contrib[p] = 0.f;
    });
    if (__ballot(alive) == 0ull) break;
    bool has = false;
    float sux = 0.f, suy = 0.f;
    f3 sC = {0.f, 0.f, 0.f};
    if (alive) {
      if (j == 0) {  // new path: vertex 0 on the emitter
        fac = emit_path(A, path, r);
        path_emitter(A, path, Le, iLe, etex);
        beta = Le * fac;
        j = 1; nrec = 0; sig = 0x811C9DC5u;
        Om = 0.f; omR = 0.f; R = 0; Sl = 0.f;
        klast = 0; vmask = 0ull;
        if (GS) {
          gs_on = false;
#pragma unroll
          for (int q = 0; q < 12; ++q) gs[q] = 0.f;
        }
      }
      Event ev = bounce<HF>(A, path, j, r, 1, stk, ss);
      if (A.sig) sig = sig_event(sig, ev);
      if (ev.kind == 1 && ev.valid) {
        f3 C = mul(beta, ev.rho) * ev.g;
        if (GS && gs_on) gs[10] += luminance(C);
        if (SPL) {
          SplatRec* o = A.spl + (size_t)(j - 1) * (size_t)A.n_paths + path;
          o->ux = ev.ux; o->uy = ev.uy; o->C[0] = C.x; o->C[1] = C.y; o->C[2] = C.z;
          klast = j; vmask |= 1ull << (j - 1);
        }
        if (!selected) { has = true; sux = ev.ux; suy = ev.uy; sC = C; }
        Sl += luminance(C);
        if (RESV) {
          float om = luminance(C);
          if (om > 0.0f) {
            Om += om;
            if (ev.u_res < om / Om) { R = j; omR = om; uxR = ev.ux; uyR = ev.uy; CR = C; }
          }
        }
      }
      if (TAPE && ev.kind != 0) {
        TapeRec t;
        if (ev.kind == 1)
          t.tf = (uint32_t)ev.texel | kTfLambert | (ev.valid ? kTfValid : 0u) | (ev.cont ? kTfScatter : 0u);
        else
          t.tf = kTfDielectric;
        t.g = ev.g; t.ux = ev.ux; t.uy = ev.uy;
        t.b[0] = beta.x; t.b[1] = beta.y; t.b[2] = beta.z; t.pad = fac;
        A.tape[(size_t)(j - 1) * (size_t)A.n_paths + path] = t;
        if (A.tape_gw) A.tape_gw[(size_t)(j - 1) * (size_t)A.n_paths + path] = ev.gw;
        LT_COUNT(8, 1);
        ++nrec;
      }
      if (ev.kind == 1 && ev.cont) beta = mul(beta, ev.rho) * ev.gw;
      if (GS && !gs_on && ev.kind == 1 && ev.cont && ev.gq > 0.f) {
        f3 na = ev.cos_in < 0.0f ? r.offn : r.offn * -1.0f;
        gs[0] = ev.x.x; gs[1] = ev.x.y; gs[2] = ev.x.z;
        gs[3] = na.x; gs[4] = na.y; gs[5] = na.z;
        gs[6] = r.w.x; gs[7] = r.w.y; gs[8] = r.w.z;
        gs[9] = ev.gq; gs[11] = (float)ev.gcomp;
        gs_on = true;
      }
      if (ev.cont) {
        ++j;
      } else {  // path finished
        if (GS)
          for (int q = 0; q < 12; ++q) A.gsamp[(size_t)path * 12 + q] = gs[q];
        float W = R > 0 ? Om / omR : 0.f;
        if (RESV && selected && R > 0) { has = true; sux = uxR; suy = uyR; sC = CR * W; }
        if (RESV && A.res) {
          ResRec rr;
          rr.R = R; rr.W = W; rr.ux = uxR; rr.uy = uyR;
          rr.S[0] = CR.x * W; rr.S[1] = CR.y * W; rr.S[2] = CR.z * W; rr.pad = 0.f;
          A.res[path] = rr;
        }
        if (TAPE) A.tape_len[path] = nrec;
        if (SPL) {
          SplatHdr hd;
          hd.klast = klast; hd.pad = 0; hd.vmask = vmask;
          A.spl_hdr[path] = hd;
        }
        if (A.sig) A.sig[path] = fnv1a(sig, (uint32_t)R);
        if (A.contrib) A.contrib[path] = Sl;
        alive = false; j = 0;
      }
    }
    if (!GS) {  // the sample pass writes no image
      keep_finite(A, has, sC);
      splat_wave(A.sc, A.image, has, sux, suy, sC);
    }
  }
}

// At most 96 VGPRs (five waves per SIMD, with the default 10 x 128-thread
// workgroups per CU), where a few registers spill: the box forward runs 3.6%
// faster than at four waves.  The plain forward with the heightfield's grid
// walk holds four (128 VGPRs, few spills): the 128x128 caustic's runs 6.7%
// faster there (5.08 -> 4.74 ms).
template <bool TAPE, bool RESV, bool SPL = false, bool GS = false, bool HF = true>
__global__ void __launch_bounds__(1024, (HF && !TAPE && !RESV && !SPL && !GS) ? 4 : 5) k_trace(PassArgs A) {
  extern __shared__ int lds[];
  trace_run<TAPE, RESV, SPL, GS, HF>(A, lds);
}

// ---------------------------------------------------------------- naive AD
// Reverse sweep over the tape, exact chain rule (no inverses, no division):
//   C_j = beta_j rho_j g_j,  beta_{j+1} = beta_j rho_j s_j (Lambertian scatter,
//   s_j = 1, or cos / (pi q) from the tape's weight array when guided),
//   beta_1 = L_e * f, with the path's emission factor f taped in every record.
// Lanes of a wave walk their tapes in lock step so that the texel
// gradients are scattered cooperatively.
__global__ void __launch_bounds__(256) k_naive_bwd(PassArgs A) {
  extern __shared__ int lds[];
  AGrad ga = agrad_begin(A, lds);
  float* le = legrad_begin(A, past_agrad(A, lds, 0));
  const size_t N = (size_t)A.n_paths;
  double gl0 = 0.0, gl1 = 0.0, gl2 = 0.0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t first = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t rounds = (N + stride - 1) / stride;
  for (size_t rd = 0; rd < rounds; ++rd) {
    size_t path = first + rd * stride;
    bool live = path < N && !(A.mask && A.mask[path] == 0);
    int k = live ? min(max(A.tape_len_in[path], 0), A.D) : 0;
    int kmax = k;
    for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
    f3 bb = {0.f, 0.f, 0.f};  // adjoint of beta_{j+1}
    float fac = 0.f;
    for (int s = 0; s < kmax; ++s) {
      int j = k - s;
      bool has = false;
      int texel = 0;
      f3 gr = {0.f, 0.f, 0.f};
      if (j >= 1) {
        TapeRec t = A.tape_in[(size_t)(j - 1) * N + path];
        LT_COUNT(9, 1);
        fac = t.pad;
        if (t.tf & kTfLambert) {  // dielectric: weight 1, adjoint passes through
          texel = min((int)(t.tf & kTexMask), A.n_texels - 1);
          f3 rho = ld3(A.albedo + (size_t)texel * 3);
          f3 b = {t.b[0], t.b[1], t.b[2]};
          f3 bj = {0.f, 0.f, 0.f};
          if (t.tf & kTfValid) {
            f3 Lb = gather(A.sc, A.dI, t.ux, t.uy);
            gr = mul(Lb, b) * t.g;
            bj = mul(Lb, rho) * t.g;
          }
          if (t.tf & kTfScatter) {
            const float sw = A.tape_gw_in ? A.tape_gw_in[(size_t)(j - 1) * N + path] : 1.0f;
            gr = gr + mul(bb, b) * sw;
            bj = bj + mul(bb, rho) * sw;
          }
          bb = bj;
          has = true;
        }
      }
      keep_finite(A, has, gr);
      scatter_albedo(A, ga, has, texel, gr);
    }
    f3 Lp = ld3(A.Le);
    if (live) {
      D3R iLp = {0.0, 0.0, 0.0};
      int etex = -1;
      path_emitter(A, (uint32_t)path, Lp, iLp, etex);
      add_le(A, gl0, gl1, gl2, (double)bb.x * fac, (double)bb.y * fac, (double)bb.z * fac, etex, le);
    }
    // the path's adjoint-weighted contribution |delta_total| = sum_c |L_e,c f bb_c|
    if (A.contrib && path < N)
      A.contrib[path] = live ? fabsf(Lp.x * fac * bb.x) + fabsf(Lp.y * fac * bb.y) + fabsf(Lp.z * fac * bb.z) : 0.f;
  }
  flush_le(A, gl0, gl1, gl2);
  agrad_end(A, ga);
  legrad_end(A, le);
}

// ---------------------------------------------------------------- ResLRB
// Replay each path up to its selected depth R and apply the log-derivative
// identity with weight w = dI(u_R) * S_hat (Eq. 11): the emitter factor
// gets w / L_e, every Lambertian factor rho_j (j < R scatter, j = R
// connection) gets w / rho_j.  No connection is re-evaluated.
__global__ void __launch_bounds__(1024) k_reslrb_bwd(PassArgs A) {
  extern __shared__ int lds[];
  int* stk = lds + threadIdx.x;
  const int ss = blockDim.x;
  AGrad ga = agrad_begin(A, lds + A.sc.stack_n * blockDim.x);
  float* le = legrad_begin(A, past_agrad(A, lds, A.sc.stack_n));
  bool alive = false, exhausted = false;
  uint32_t path = 0;
  int j = 0, R = 0;
  Ray r;
  f3 w = {0.f, 0.f, 0.f};
  f3 Le = ld3(A.Le);
  D3R iLe = recip_le(Le);
  int etex = -1;
  double gl0 = 0.0, gl1 = 0.0, gl2 = 0.0;
  WorkQ wq = work_begin(A.counter);
  while (true) {
    refill(A, wq, alive, exhausted, path, [&](uint32_t) {});
    if (__ballot(alive) == 0ull) break;
    bool has = false;
    int texel = 0;
    f3 gv = {0.f, 0.f, 0.f};
    if (alive && j == 0) {
      ResRec rec = A.res_in[path];
      if (rec.R <= 0) {
        alive = false;
      } else {
        R = min(rec.R, A.D);
        f3 Lb = gather(A.sc, A.dI, rec.ux, rec.uy);
        w = mul(Lb, mk(rec.S[0], rec.S[1], rec.S[2]));
        path_emitter(A, path, Le, iLe, etex);
        add_le(A, gl0, gl1, gl2, (double)w.x * iLe.x, (double)w.y * iLe.y, (double)w.z * iLe.z, etex, le);
        emit_path(A, path, r);
        j = 1;
      }
    }
    if (alive) {
      Event ev = bounce(A, path, j, r, 0, stk, ss);
      if (ev.kind == 1) {
        texel = ev.texel;
        gv = {ev.rho.x > 0.f ? w.x / ev.rho.x : 0.f, ev.rho.y > 0.f ? w.y / ev.rho.y : 0.f,
              ev.rho.z > 0.f ? w.z / ev.rho.z : 0.f};
        has = true;
      }
      if (ev.cont && j < R) ++j;
      else { alive = false; j = 0; }
    }
    keep_finite(A, has, gv);
    scatter_albedo(A, ga, has, texel, gv);
  }
  flush_le(A, gl0, gl1, gl2);
  agrad_end(A, ga);
  legrad_end(A, le);
}

// ---------------------------------------------------------------- LRB-3
// Pass 2 and Pass 3 fused per path (dI is read-only between them):
// phase 2 replays and accumulates delta_total = sum_i dI(u_i) * C_i
// (Eq. 14, FP64); phase 3 replays again: the splat term dI(u_i) * C_i / rho_i
// (Eq. 15), the subtraction delta_rem -= dI(u_i) * C_i (Eq. 16) and the
// log-derivative delta_rem / rho_i of the scatter factor (Eq. 17); the
// emitter gets delta_total / L_e.
// Phase 2 also keeps one bit per vertex (valid connection) and the depth of
// the last valid connection: phase 3 then re-evaluates only the connection
// geometry where the bit is set (no shadow rays) and stops at that depth,
// where delta_rem is exactly zero and nothing further contributes.
template <bool HF = true>
__device__ __forceinline__ void lrb3_run(const PassArgs& A, int* lds) {
  int* stk = lds + threadIdx.x;
  const int ss = blockDim.x;
  AGrad ga = agrad_begin(A, lds + A.sc.stack_n * blockDim.x);
  float* le = legrad_begin(A, past_agrad(A, lds, A.sc.stack_n));
  bool alive = false, exhausted = false;
  uint32_t path = 0;
  int j = 0, phase = 2, klast = 0;
  uint64_t vmask = 0ull;
  Ray r;
  f3 beta = {0.f, 0.f, 0.f};
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;  // delta_total, then delta_rem
  f3 Le = ld3(A.Le);
  D3R iLe = recip_le(Le);
  int etex = -1;
  double gl0 = 0.0, gl1 = 0.0, gl2 = 0.0;
  WorkQ wq = work_begin(A.counter);
  while (true) {
    refill(A, wq, alive, exhausted, path, [&](uint32_t p) { if (A.contrib) A.contrib[p] = 0.f; });
    if (__ballot(alive) == 0ull) break;
    bool has = false;
    int texel = 0;
    f3 gv = {0.f, 0.f, 0.f};
    if (alive) {
      if (j == 0) {
        float f = emit_path(A, path, r);
        path_emitter(A, path, Le, iLe, etex);
        beta = Le * f;
        j = 1;
        if (phase == 2) { d0 = d1 = d2 = 0.0; vmask = 0ull; klast = 0; }
      }
      const int cmode = phase == 2 ? 1 : (((vmask >> (j - 1)) & 1ull) ? 2 : 0);
      Event ev = bounce<HF>(A, path, j, r, cmode, stk, ss);
      if (phase == 3 && j >= klast) ev.cont = false;  // nothing after the last connection
      if (ev.kind == 1) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        if (ev.valid) {
          f3 C = mul(beta, ev.rho) * ev.g;
          f3 Lb = gather(A.sc, A.dI, ev.ux, ev.uy);
          a0 = (double)Lb.x * C.x; a1 = (double)Lb.y * C.y; a2 = (double)Lb.z * C.z;
          if (phase == 2) { vmask |= 1ull << (j - 1); klast = j; }
        }
        if (phase == 2) {
          d0 += a0; d1 += a1; d2 += a2;
        } else {
          d0 -= a0; d1 -= a1; d2 -= a2;
          if (j >= klast) { d0 = d1 = d2 = 0.0; }
          double g0 = a0, g1 = a1, g2 = a2;
          if (ev.cont) { g0 += d0; g1 += d1; g2 += d2; }
          texel = ev.texel;
          gv = {ev.rho.x > 0.f ? (float)g0 / ev.rho.x : 0.f, ev.rho.y > 0.f ? (float)g1 / ev.rho.y : 0.f,
                ev.rho.z > 0.f ? (float)g2 / ev.rho.z : 0.f};
          has = true;
        }
        if (ev.cont) beta = mul(beta, ev.rho) * ev.gw;
      }
      if (ev.cont) {
        ++j;
      } else if (phase == 2 && klast > 0 && (d0 != 0.0 || d1 != 0.0 || d2 != 0.0)) {  // consuming replay
        add_le(A, gl0, gl1, gl2, d0 * iLe.x, d1 * iLe.y, d2 * iLe.z, etex, le);
        // the path's adjoint-weighted contribution |delta_total|
        if (A.contrib) A.contrib[path] = (float)(fabs(d0) + fabs(d1) + fabs(d2));
        phase = 3; j = 0;
      } else {
        if (A.contrib && phase == 2) A.contrib[path] = 0.f;
        phase = 2; j = 0; alive = false;
      }
    }
    keep_finite(A, has, gv);
    scatter_albedo(A, ga, has, texel, gv);
  }
  flush_le(A, gl0, gl1, gl2);
  agrad_end(A, ga);
  legrad_end(A, le);
  lds_grads_done(A);
}

// HF = false: the instantiation for scenes without a heightfield
template <bool HF>
__global__ void __launch_bounds__(1024) k_lrb3_bwd(PassArgs A) {
  extern __shared__ int lds[];
  lrb3_run<HF>(A, lds);
}

// ---------------------------------------------------------------- buffered two-pass
// The buffered two-pass variant (lrb_2pass, Sec. 4.1 and Sec. 6): the forward
// stored every connection's film position and contribution in a buffer
// preallocated to the maximum depth, so delta_total = sum_i dI(u_i) C_i
// (Eq. 14) is read back without a traversal, and one replay (no shadow rays,
// no connection geometry: u_i and C_i come from the buffer) consumes it as
// LRB-3's pass 3 does (Eq. 15-17).  Memory is linear in depth, traversals
// two (forward and replay), the gradient naive AD's.
__device__ __forceinline__ void lrb2_run(const PassArgs& A, int* lds) {
  int* stk = lds + threadIdx.x;
  const int ss = blockDim.x;
  AGrad ga = agrad_begin(A, lds + A.sc.stack_n * blockDim.x);
  float* le = legrad_begin(A, past_agrad(A, lds, A.sc.stack_n));
  const size_t N = (size_t)A.n_paths;
  bool alive = false, exhausted = false;
  uint32_t path = 0;
  int j = 0, klast = 0;
  uint64_t vmask = 0ull;
  Ray r;
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  f3 Le = ld3(A.Le);
  D3R iLe = recip_le(Le);
  int etex = -1;
  double gl0 = 0.0, gl1 = 0.0, gl2 = 0.0;
  WorkQ wq = work_begin(A.counter);
  while (true) {
    refill(A, wq, alive, exhausted, path, [&](uint32_t p) { if (A.contrib) A.contrib[p] = 0.f; });
    if (__ballot(alive) == 0ull) break;
    bool has = false;
    int texel = 0;
    f3 gv = {0.f, 0.f, 0.f};
    if (alive && j == 0) {
      const SplatHdr hd = A.spl_hdr_in[path];
      klast = min(hd.klast, A.D);
      vmask = hd.vmask;
      d0 = d1 = d2 = 0.0;
      for (uint64_t m = vmask; m; m &= m - 1ull) {
        const int i = __ffsll((unsigned long long)m);  // 1-based vertex
        if (i > klast) break;
        const SplatRec rec = A.spl_in[(size_t)(i - 1) * N + path];
        LT_COUNT(9, 1);
        f3 Lb = gather(A.sc, A.dI, rec.ux, rec.uy);
        d0 += (double)Lb.x * rec.C[0]; d1 += (double)Lb.y * rec.C[1]; d2 += (double)Lb.z * rec.C[2];
      }
      if (klast > 0 && (d0 != 0.0 || d1 != 0.0 || d2 != 0.0)) {
        path_emitter(A, path, Le, iLe, etex);
        add_le(A, gl0, gl1, gl2, d0 * iLe.x, d1 * iLe.y, d2 * iLe.z, etex, le);
        if (A.contrib) A.contrib[path] = (float)(fabs(d0) + fabs(d1) + fabs(d2));
        emit_path(A, path, r);
        j = 1;
      } else {
        if (A.contrib) A.contrib[path] = 0.f;
        alive = false;
      }
    }
    if (alive) {
      Event ev = bounce(A, path, j, r, 0, stk, ss);
      const bool last = j >= klast;
      if (ev.kind == 1) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        if ((vmask >> (j - 1)) & 1ull) {
          const SplatRec rec = A.spl_in[(size_t)(j - 1) * N + path];
          LT_COUNT(9, 1);
          f3 Lb = gather(A.sc, A.dI, rec.ux, rec.uy);
          a0 = (double)Lb.x * rec.C[0]; a1 = (double)Lb.y * rec.C[1]; a2 = (double)Lb.z * rec.C[2];
        }
        d0 -= a0; d1 -= a1; d2 -= a2;
        if (last) { d0 = d1 = d2 = 0.0; }
        double g0 = a0, g1 = a1, g2 = a2;
        if (!last) { g0 += d0; g1 += d1; g2 += d2; }
        texel = ev.texel;
        gv = {ev.rho.x > 0.f ? (float)g0 / ev.rho.x : 0.f, ev.rho.y > 0.f ? (float)g1 / ev.rho.y : 0.f,
              ev.rho.z > 0.f ? (float)g2 / ev.rho.z : 0.f};
        has = true;
      }
      if (ev.cont && !last) ++j;
      else { alive = false; j = 0; }
    }
    keep_finite(A, has, gv);
    scatter_albedo(A, ga, has, texel, gv);
  }
  flush_le(A, gl0, gl1, gl2);
  agrad_end(A, ga);
  legrad_end(A, le);
}

__global__ void __launch_bounds__(1024) k_lrb2_bwd(PassArgs A) {
  extern __shared__ int lds[];
  lrb2_run(A, lds);
}

// ---------------------------------------------------------------- LRB-3, two kernels
// The same two replays as k_lrb3_bwd, each a kernel of its own with the
// method's per-path state handed over in memory (Lrb3Hand, 40 bytes per
// connected path, appended per class of the path index, flat in depth).
// Every wave then runs one phase: pass 2's shadow rays and pass 3's gradient
// scatters never share a wave, and pass 3 visits only the paths with a
// sensor connection, compacted by the append.

// Pass 2 (Eq. 14): replay with the sensor connections (shadow rays
// included), delta_total = sum_i dI(u_i) C_i in FP64, one bit per vertex for
// a valid connection, the depth of the last one.  A path whose delta_total is
// nonzero gets its emitter gradient delta_total / L_e here and a hand-off
// entry (appended to its class's region).
__device__ __forceinline__ void lrb3_p2_run(const PassArgs& A, int* lds) {
  int* stk = lds + threadIdx.x;
  const int ss = blockDim.x;
  float* le = legrad_begin(A, past_agrad(A, lds, A.sc.stack_n));
  bool alive = false, exhausted = false;
  uint32_t path = 0;
  int j = 0, klast = 0;
  uint64_t vmask = 0ull;
  Ray r;
  f3 beta = {0.f, 0.f, 0.f};
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  f3 Le = ld3(A.Le);
  D3R iLe = recip_le(Le);
  int etex = -1;
  double gl0 = 0.0, gl1 = 0.0, gl2 = 0.0;
  WorkQ wq = work_begin(A.counter);
  while (true) {
    refill(A, wq, alive, exhausted, path, [&](uint32_t p) { if (A.contrib) A.contrib[p] = 0.f; });
    if (__ballot(alive) == 0ull) break;
    bool put = false;
    if (alive) {
      if (j == 0) {
        const float f = emit_path(A, path, r);
        path_emitter(A, path, Le, iLe, etex);
        beta = Le * f;
        j = 1;
        d0 = d1 = d2 = 0.0; vmask = 0ull; klast = 0;
      }
      Event ev = bounce(A, path, j, r, 1, stk, ss);
      if (ev.kind == 1) {
        if (ev.valid) {
          f3 C = mul(beta, ev.rho) * ev.g;
          f3 Lb = gather(A.sc, A.dI, ev.ux, ev.uy);
          d0 += (double)Lb.x * C.x; d1 += (double)Lb.y * C.y; d2 += (double)Lb.z * C.z;
          vmask |= 1ull << (j - 1); klast = j;
        }
        if (ev.cont) beta = mul(beta, ev.rho) * ev.gw;
      }
      if (ev.cont) {
        ++j;
      } else {
        put = klast > 0 && (d0 != 0.0 || d1 != 0.0 || d2 != 0.0);
        if (put) add_le(A, gl0, gl1, gl2, d0 * iLe.x, d1 * iLe.y, d2 * iLe.z, etex, le);
        // the path's adjoint-weighted contribution |delta_total|
        if (A.contrib) A.contrib[path] = put ? (float)(fabs(d0) + fabs(d1) + fabs(d2)) : 0.f;
        alive = false; j = 0;
      }
    }
    const uint32_t slot = hand_append(A, put, path);
    if (put) {
      Lrb3Hand h;
      h.path = path; h.klast = klast; h.vmask = vmask; h.d[0] = d0; h.d[1] = d1; h.d[2] = d2;
      A.hand[slot] = h;
    }
  }
  flush_le(A, gl0, gl1, gl2);
  legrad_end(A, le);
}

// Pass 3 (Eq. 15-17) over the handed-over paths: replay to the last
// connection re-evaluating only the connection geometry where the bit is
// set (no shadow rays), the splat term dI(u_i) C_i / rho_i, the subtraction
// from delta_rem and the scatter term delta_rem / rho_i.
__device__ __forceinline__ void lrb3_p3_run(const PassArgs& A, int* lds) {
  int* stk = lds + threadIdx.x;
  const int ss = blockDim.x;
  AGrad ga = agrad_begin(A, lds + A.sc.stack_n * blockDim.x);
  bool alive = false, exhausted = false;
  uint32_t item = 0, path = 0;
  int j = 0, klast = 0;
  uint64_t vmask = 0ull;
  Ray r;
  f3 beta = {0.f, 0.f, 0.f};
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  f3 Le = ld3(A.Le);
  D3R iLe = {0.0, 0.0, 0.0};
  int etex = -1;
  WorkQ wq = work_begin(A.counter3);
  while (true) {
    refill_hand(A, wq, alive, exhausted, item);
    if (__ballot(alive) == 0ull) break;
    bool has = false;
    int texel = 0;
    f3 gv = {0.f, 0.f, 0.f};
    if (alive) {
      if (j == 0) {
        const Lrb3Hand h = A.hand[item];
        path = h.path; klast = h.klast; vmask = h.vmask; d0 = h.d[0]; d1 = h.d[1]; d2 = h.d[2];
        const float f = emit_path(A, path, r);
        path_emitter(A, path, Le, iLe, etex);
        beta = Le * f;
        j = 1;
      }
      Event ev = bounce(A, path, j, r, ((vmask >> (j - 1)) & 1ull) ? 2 : 0, stk, ss);
      if (j >= klast) ev.cont = false;  // nothing after the last connection
      if (ev.kind == 1) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        if (ev.valid) {
          f3 C = mul(beta, ev.rho) * ev.g;
          f3 Lb = gather(A.sc, A.dI, ev.ux, ev.uy);
          a0 = (double)Lb.x * C.x; a1 = (double)Lb.y * C.y; a2 = (double)Lb.z * C.z;
        }
        d0 -= a0; d1 -= a1; d2 -= a2;
        if (j >= klast) { d0 = d1 = d2 = 0.0; }
        double g0 = a0, g1 = a1, g2 = a2;
        if (ev.cont) { g0 += d0; g1 += d1; g2 += d2; }
        texel = ev.texel;
        gv = {ev.rho.x > 0.f ? (float)g0 / ev.rho.x : 0.f, ev.rho.y > 0.f ? (float)g1 / ev.rho.y : 0.f,
              ev.rho.z > 0.f ? (float)g2 / ev.rho.z : 0.f};
        has = true;
        if (ev.cont) beta = mul(beta, ev.rho) * ev.gw;
      }
      if (ev.cont) ++j;
      else { alive = false; j = 0; }
    }
    keep_finite(A, has, gv);
    scatter_albedo(A, ga, has, texel, gv);
  }
  agrad_end(A, ga);
}

__global__ void __launch_bounds__(1024) k_lrb3_p2(PassArgs A) {
  extern __shared__ int lds[];
  lrb3_p2_run(A, lds);
}
__global__ void __launch_bounds__(1024) k_lrb3_p3(PassArgs A) {
  extern __shared__ int lds[];
  lrb3_p3_run(A, lds);
}

// ---------------------------------------------------------------- small kernels
__global__ void k_fill_f32(float* p, size_t n, float v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u32(unsigned int* p, size_t n, unsigned int v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f64(double* p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_add_f64_to_f32(const double* src, float* dst, int n) {
  int i = threadIdx.x;
  if (i < n && dst) dst[i] += (float)src[i];
}

__global__ void __launch_bounds__(256) k_loss(const float* I, const float* T, size_t n, float* dI, double* acc) {
  double s = 0.0;
  const double inv = 1.0 / (double)n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double d = (double)I[i] - (double)T[i];
    s += d * d;
    dI[i] = (float)(2.0 * d * inv);
  }
  s = wave_sum(s);
  __shared__ double part[16];
  int wv = threadIdx.x >> 6;
  if (__lane_id() == 0) part[wv] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += part[k];
    atomicAdd(acc, t);
  }
}
__global__ void k_loss_finish(const double* acc, size_t n, float* loss) { loss[0] = (float)(acc[0] / (double)n); }

// Heightfield triangles from the current heights, written at their BVH slots.
// The edges are built from height differences and whole grid steps, not by
// subtracting rounded corner positions: base + h rounds to about 6e-8 at
// base 0.6, which on a 1/127 grid spacing would put ~1e-5 of error on every
// facet slope, whereas h_k - h_0 and (i_k - i_0) dx are exact or nearly so.
__global__ void k_hf_tris(DevScene sc, Tri* tris, const float* h) {
  int nhf = 2 * (sc.hf_G - 1) * (sc.hf_G - 1);
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nhf) return;
  int gi[3], gj[3];
  float hv[3];
  for (int k = 0; k < 3; ++k) {
    hf_corner(sc.hf_G, q, k, gi[k], gj[k]);
    hv[k] = hget(h, sc.hf_G, gi[k], gj[k]);
  }
  Tri t;
  t.p0[0] = sc.hf_x0 + gi[0] * sc.hf_dx;
  t.p0[1] = sc.hf_base + hv[0];
  t.p0[2] = sc.hf_z0 + gj[0] * sc.hf_dx;
  t.prim = sc.n_static + q;
  t.e1[0] = (float)(gi[1] - gi[0]) * sc.hf_dx; t.e1[1] = hv[1] - hv[0]; t.e1[2] = (float)(gj[1] - gj[0]) * sc.hf_dx;
  t.e2[0] = (float)(gi[2] - gi[0]) * sc.hf_dx; t.e2[1] = hv[2] - hv[0]; t.e2[2] = (float)(gj[2] - gj[0]) * sc.hf_dx;
  t.pad1 = 0.f; t.pad2 = 0.f;
  tris[sc.n_static + q] = t;  // the heightfield's slots follow the static triangles
}

// least and greatest height into hb[0], hb[1] (one workgroup of 1024)
__global__ void __launch_bounds__(1024) k_hf_bounds(const float* h, int n, float* hb) {
  __shared__ float lo[1024], hi[1024];
  float a = 3.0e38f, b = -3.0e38f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) { a = fminf(a, h[i]); b = fmaxf(b, h[i]); }
  lo[threadIdx.x] = a; hi[threadIdx.x] = b;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + w]);
      hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { hb[0] = lo[0]; hb[1] = hi[0]; }
}

#include "lt_attached.inc"
#include "lt_camera.inc"

// ---------------------------------------------------------------- batches
// One persistent launch over a table of instances (scenes, films, path
// counts and depths of their own).  Every wave walks the table in order and
// takes work tickets (path indices) from each instance's own counter; a wave
// moves on once its lanes have drained an instance, so an instance's
// arguments stay uniform across the wave and the cooperative splat and
// gradient scatter work unchanged.  Waves that finish an instance early start
// on the next one while others drain: no launch gaps, one tail per launch.
// Pointers read from ordinary memory are generic to the compiler, so every
// access through them would be a flat instruction (address-space check,
// counted on both the vector-memory and LDS counters).  The table is
// read-only during a launch and is read through the constant address space,
// as kernel arguments are; pointers loaded from there are taken to be global
// memory, and loads, stores and atomics through them compile to global ones.
__device__ __forceinline__ PassArgs table_entry(const PassArgs* T, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
  return ((const __attribute__((address_space(4))) PassArgs*)T)[i];
#else
  return T[i];  // host pass of the device function: never executed
#endif
}

__global__ void __launch_bounds__(1024) k_trace_batch(const PassArgs* __restrict__ T, int n) {
  extern __shared__ int lds[];
  for (int i = 0; i < n; ++i) trace_run<false, false>(table_entry(T, i), lds);
}
// One table entry through the single-instance forward, at its register
// budget (five waves per SIMD without the heightfield walk, four with it),
// without the walk where the scene has none.  Batches run their largest
// instances' forwards through it.
template <bool HF>
__global__ void __launch_bounds__(1024, HF ? 4 : 5) k_trace_entry(const PassArgs* __restrict__ T) {
  extern __shared__ int lds[];
  trace_run<false, false, false, false, HF>(table_entry(T, 0), lds);
}
// HF = false: no entry's scene has a heightfield
template <bool HF>
__global__ void __launch_bounds__(1024) k_lrb3_batch(const PassArgs* __restrict__ T, int n) {
  extern __shared__ int lds[];
  for (int i = 0; i < n; ++i) lrb3_run<HF>(table_entry(T, i), lds);
}
// One detached entry of the table as the single-instance kernel runs it:
// without the loop over entries, which holds live state across the
// instances and costs the multi-entry kernel spill space (140 against 60
// bytes per lane).  Batches run their large detached instances through it.
template <bool HF>
__global__ void __launch_bounds__(1024) k_lrb3_entry(const PassArgs* __restrict__ T) {
  extern __shared__ int lds[];
  lrb3_run<HF>(table_entry(T, 0), lds);
}
__global__ void __launch_bounds__(256, 2) k_lrb3_att_batch(const PassArgs* __restrict__ T, int n) {
  extern __shared__ int lds[];
  for (int i = 0; i < n; ++i) lrb3_att_run<false>(table_entry(T, i), lds);
}
// One attached entry of the table, at the single-instance kernel's three
// waves per SIMD and workgroup sizes (the loop over entries above costs
// registers enough to hold that kernel to two).  Batches run their large
// attached instances through it, one launch each; the arguments stay in the
// table, so a replayed graph reads each step's seeds.
__global__ void __launch_bounds__(768, 3) k_lrb3_att_entry(const PassArgs* __restrict__ T) {
  extern __shared__ int lds[];
  lrb3_att_run<false>(table_entry(T, 0), lds);
}

// The two-kernel attached LRB-3 reading one table entry: batches run their
// large attached instances through this pair, as the single-instance call
// does (the hand-off buffer and pass 3's counters are in the entry).
__global__ void __launch_bounds__(768, 3) k_lrb3_att_p2_entry(const PassArgs* __restrict__ T) {
  extern __shared__ int lds[];
  lrb3_att_p2_run<false>(table_entry(T, 0), lds);
}
__global__ void __launch_bounds__(768, 3) k_lrb3_att_p3_entry(const PassArgs* __restrict__ T) {
  extern __shared__ int lds[];
  lrb3_att_p3_run<false>(table_entry(T, 0), lds);
}

#ifdef LT_COUNTERS
}  // namespace counted
#endif

// ---------------------------------------------------------------- launchers
static size_t stack_bytes(const PassArgs& A, int block) { return (size_t)A.sc.stack_n * block * sizeof(int); }
static size_t hgrad_bytes(const PassArgs& A) {
  return A.hgrad_lds ? (size_t)A.sc.hf_G * A.sc.hf_G * sizeof(float) : 0;
}
static size_t agrad_bytes(const PassArgs& A) { return A.agrad_lds ? (size_t)A.n_texels * 3 * sizeof(float) : 0; }
static size_t legrad_bytes(const PassArgs& A) {
  return A.legrad_lds ? (size_t)A.sc.em_tex_res * A.sc.em_tex_res * 3 * sizeof(float) : 0;
}

// allow the backward kernels the device's full LDS per workgroup
hipError_t set_lds_limit(int bytes) {
  hipError_t e = hipSuccess;
  for (const void* f : {(const void*)k_lrb3_att<false>, (const void*)k_lrb3_att<true>, (const void*)k_reslrb_att<false>,
                        (const void*)k_reslrb_att<true>, (const void*)k_naive_att_bwd<false>,
                        (const void*)k_naive_att_bwd<true>})
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  for (const void* f : {(const void*)k_lrb3_bwd<true>, (const void*)k_lrb3_bwd<false>})
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_reslrb_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_naive_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  for (const void* f : {(const void*)k_lrb3_batch<true>, (const void*)k_lrb3_batch<false>,
                        (const void*)k_lrb3_entry<true>, (const void*)k_lrb3_entry<false>})
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_lrb3_att_batch, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_lrb3_att_entry, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  for (const void* f : {(const void*)k_lrb3_att_p2_entry, (const void*)k_lrb3_att_p3_entry,
                        (const void*)k_lrb3_p2, (const void*)k_lrb3_p3, (const void*)k_lrb3_att_p2<false>,
                        (const void*)k_lrb3_att_p3<false>, (const void*)k_lrb3_att_p2<true>,
                        (const void*)k_lrb3_att_p3<true>, (const void*)k_lrb2_bwd, (const void*)k_camera_prb})
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}

int resident_groups(BwdKernel k, int block, size_t lds) {
  // the answer depends only on the arguments and the device: cache it
  static std::mutex mu;
  static std::map<std::tuple<int, int, int, size_t>, int> memo;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) (void)hipGetLastError();
  const auto key = std::make_tuple(dev, (int)k, block, lds);
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
  }
  const void* f = nullptr;
  switch (k) {
    case BwdKernel::naive: f = (const void*)k_naive_bwd; break;
    case BwdKernel::reslrb: f = (const void*)k_reslrb_bwd; break;
    case BwdKernel::lrb3: f = (const void*)k_lrb3_bwd<true>; break;
    case BwdKernel::naive_att: f = (const void*)k_naive_att_bwd<false>; break;
    case BwdKernel::reslrb_att: f = (const void*)k_reslrb_att<false>; break;
    case BwdKernel::lrb3_att: f = (const void*)k_lrb3_att<false>; break;
    case BwdKernel::lrb3_batch: f = (const void*)k_lrb3_batch<true>; break;
    case BwdKernel::lrb3_entry: f = (const void*)k_lrb3_entry<true>; break;
    case BwdKernel::lrb3_att_p3_cond: f = (const void*)k_lrb3_att_p3<true>; break;
    case BwdKernel::lrb3_att_cond: f = (const void*)k_lrb3_att<true>; break;
    case BwdKernel::lrb3_att_batch: f = (const void*)k_lrb3_att_batch; break;
    case BwdKernel::lrb3_att_entry: f = (const void*)k_lrb3_att_entry; break;
    case BwdKernel::lrb3_att_p3_entry: f = (const void*)k_lrb3_att_p3_entry; break;
    case BwdKernel::lrb3_p2: f = (const void*)k_lrb3_p2; break;
    case BwdKernel::lrb3_p3: f = (const void*)k_lrb3_p3; break;
    case BwdKernel::lrb3_att_p2: f = (const void*)k_lrb3_att_p2<false>; break;
    case BwdKernel::lrb3_att_p3: f = (const void*)k_lrb3_att_p3<false>; break;
    case BwdKernel::lrb2: f = (const void*)k_lrb2_bwd; break;
    case BwdKernel::camera_prb: f = (const void*)k_camera_prb; break;
  }
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, block, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  std::lock_guard<std::mutex> g(mu);
  memo[key] = n;
  return n;
}

hipError_t launch_lrb3_att(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(A.cond ? k_lrb3_att<true> : k_lrb3_att<false>, dim3(grid), dim3(block), stack_bytes(A, block) + hgrad_bytes(A) + agrad_bytes(A), s,
                     A);
  return hipGetLastError();
}
hipError_t launch_trace_att(const PassArgs& A, bool tape, bool resv, int grid, hipStream_t s) {
  size_t sh = stack_bytes(A, 256);
  if (tape && resv && A.cond) hipLaunchKernelGGL((k_trace_att<true, true, true>), dim3(grid), dim3(256), sh, s, A);
  else if (tape && resv) hipLaunchKernelGGL((k_trace_att<true, true>), dim3(grid), dim3(256), sh, s, A);
  else if (tape && A.cond) hipLaunchKernelGGL((k_trace_att<true, false, true>), dim3(grid), dim3(256), sh, s, A);
  else if (tape) hipLaunchKernelGGL((k_trace_att<true, false>), dim3(grid), dim3(256), sh, s, A);
  else if (A.cond) hipLaunchKernelGGL((k_trace_att<false, true, true>), dim3(grid), dim3(256), sh, s, A);
  else hipLaunchKernelGGL((k_trace_att<false, true>), dim3(grid), dim3(256), sh, s, A);
  return hipGetLastError();
}
hipError_t launch_naive_att_bwd(const PassArgs& A, int grid, hipStream_t s) {
  hipLaunchKernelGGL(A.cond ? k_naive_att_bwd<true> : k_naive_att_bwd<false>, dim3(grid), dim3(256), hgrad_bytes(A) + agrad_bytes(A), s, A);
  return hipGetLastError();
}
hipError_t launch_reslrb_att(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(A.cond ? k_reslrb_att<true> : k_reslrb_att<false>, dim3(grid), dim3(block), stack_bytes(A, block) + hgrad_bytes(A) + agrad_bytes(A), s,
                     A);
  return hipGetLastError();
}

hipError_t launch_trace_batch(const PassArgs* table, int n, int stack_n, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_trace_batch, dim3(grid), dim3(block), (size_t)stack_n * block * sizeof(int), s, table, n);
  return hipGetLastError();
}
hipError_t launch_trace_entry(const PassArgs* entry, bool hf, int stack_n, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(hf ? k_trace_entry<true> : k_trace_entry<false>, dim3(grid), dim3(block),
                     (size_t)stack_n * block * sizeof(int), s, entry);
  return hipGetLastError();
}
hipError_t launch_lrb3_batch(const PassArgs* table, int n, bool hf, int stack_n, size_t grad_lds, int grid, int block,
                             hipStream_t s) {
  hipLaunchKernelGGL(hf ? k_lrb3_batch<true> : k_lrb3_batch<false>, dim3(grid), dim3(block),
                     (size_t)stack_n * block * sizeof(int) + grad_lds, s, table, n);
  return hipGetLastError();
}
hipError_t launch_lrb3_entry(const PassArgs* entry, bool hf, int stack_n, size_t grad_lds, int grid, int block,
                             hipStream_t s) {
  hipLaunchKernelGGL(hf ? k_lrb3_entry<true> : k_lrb3_entry<false>, dim3(grid), dim3(block),
                     (size_t)stack_n * block * sizeof(int) + grad_lds, s, entry);
  return hipGetLastError();
}
hipError_t launch_lrb3_att_batch(const PassArgs* table, int n, int stack_n, size_t grad_lds, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_lrb3_att_batch, dim3(grid), dim3(256), (size_t)stack_n * 256 * sizeof(int) + grad_lds, s, table,
                     n);
  return hipGetLastError();
}
hipError_t launch_lrb3_att_entry(const PassArgs* entry, int stack_n, size_t grad_lds, int grid, int block,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_lrb3_att_entry, dim3(grid), dim3(block), (size_t)stack_n * block * sizeof(int) + grad_lds, s,
                     entry);
  return hipGetLastError();
}
hipError_t launch_lrb3_att_split_entry(const PassArgs* entry, int stack_n, size_t grad_lds, int grid2, int grid3,
                                      int block3, hipStream_t s) {
  const size_t st2 = (size_t)stack_n * 256 * sizeof(int), st3 = (size_t)stack_n * block3 * sizeof(int);
  hipLaunchKernelGGL(k_lrb3_att_p2_entry, dim3(grid2), dim3(256), st2, s, entry);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lrb3_att_p3_entry, dim3(grid3), dim3(block3), st3 + grad_lds, s, entry);
  return hipGetLastError();
}

hipError_t read_counters(uint64_t* out, bool reset, hipStream_t s) {
#ifdef LT_COUNTERS
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  e = hipMemcpyFromSymbol(out, HIP_SYMBOL(lt_counters), 16 * sizeof(uint64_t), 0, hipMemcpyDeviceToHost);
  if (e != hipSuccess || !reset) return e;
  uint64_t z[16] = {0};
  return hipMemcpyToSymbol(HIP_SYMBOL(lt_counters), z, sizeof(z), 0, hipMemcpyHostToDevice);
#else
  (void)out; (void)reset; (void)s;
  return hipErrorNotSupported;
#endif
}

hipError_t launch_trace(const PassArgs& A, bool tape, bool resv, int grid, int block, hipStream_t s) {
  size_t sh = stack_bytes(A, block);
  if (tape && resv) hipLaunchKernelGGL((k_trace<true, true>), dim3(grid), dim3(block), sh, s, A);
  else if (tape) hipLaunchKernelGGL((k_trace<true, false>), dim3(grid), dim3(block), sh, s, A);
  else if (resv) hipLaunchKernelGGL((k_trace<false, true>), dim3(grid), dim3(block), sh, s, A);
  else if (A.sc.hf_G >= 2) hipLaunchKernelGGL((k_trace<false, false>), dim3(grid), dim3(block), sh, s, A);
  else hipLaunchKernelGGL((k_trace<false, false, false, false, false>), dim3(grid), dim3(block), sh, s, A);
  return hipGetLastError();
}

hipError_t launch_camera(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_camera, dim3(grid), dim3(block), stack_bytes(A, block), s, A);
  return hipGetLastError();
}
hipError_t launch_camera_prb(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_camera_prb, dim3(grid), dim3(block), stack_bytes(A, block) + agrad_bytes(A), s, A);
  return hipGetLastError();
}

hipError_t launch_naive_bwd(const PassArgs& A, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_naive_bwd, dim3(grid), dim3(256), agrad_bytes(A) + legrad_bytes(A), s, A);
  return hipGetLastError();
}

hipError_t launch_reslrb_bwd(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_reslrb_bwd, dim3(grid), dim3(block), stack_bytes(A, block) + agrad_bytes(A) + legrad_bytes(A), s,
                     A);
  return hipGetLastError();
}

hipError_t launch_lrb3_bwd(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(A.sc.hf_G >= 2 ? k_lrb3_bwd<true> : k_lrb3_bwd<false>, dim3(grid), dim3(block),
                     stack_bytes(A, block) + agrad_bytes(A) + legrad_bytes(A), s, A);
  return hipGetLastError();
}

hipError_t launch_trace_splats(const PassArgs& A, bool resv, int grid, int block, hipStream_t s) {
  size_t sh = stack_bytes(A, block);
  if (resv) hipLaunchKernelGGL((k_trace<false, true, true>), dim3(grid), dim3(block), sh, s, A);
  else hipLaunchKernelGGL((k_trace<false, false, true>), dim3(grid), dim3(block), sh, s, A);
  return hipGetLastError();
}
hipError_t launch_trace_gsamples(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL((k_trace<false, false, false, true>), dim3(grid), dim3(block), stack_bytes(A, block), s, A);
  return hipGetLastError();
}
hipError_t launch_lrb2_bwd(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_lrb2_bwd, dim3(grid), dim3(block), stack_bytes(A, block) + agrad_bytes(A) + legrad_bytes(A), s,
                     A);
  return hipGetLastError();
}

hipError_t launch_lrb3_p2(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_lrb3_p2, dim3(grid), dim3(block), stack_bytes(A, block) + agrad_bytes(A) + legrad_bytes(A), s,
                     A);
  return hipGetLastError();
}
hipError_t launch_lrb3_p3(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_lrb3_p3, dim3(grid), dim3(block), stack_bytes(A, block) + agrad_bytes(A), s, A);
  return hipGetLastError();
}
hipError_t launch_lrb3_att_p2(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(A.cond ? k_lrb3_att_p2<true> : k_lrb3_att_p2<false>, dim3(grid), dim3(block), stack_bytes(A, block), s, A);
  return hipGetLastError();
}
hipError_t launch_lrb3_att_p3(const PassArgs& A, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL(A.cond ? k_lrb3_att_p3<true> : k_lrb3_att_p3<false>, dim3(grid), dim3(block), stack_bytes(A, block) + hgrad_bytes(A) + agrad_bytes(A),
                     s, A);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_fill_f32, dim3(grid), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u32(unsigned int* p, size_t n, unsigned int v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_fill_f64, dim3(grid), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_add_le(const double* acc, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f64_to_f32, dim3(1), dim3(64), 0, s, acc, dst, 3);
  return hipGetLastError();
}
hipError_t launch_loss(const float* I, const float* T, size_t n, float* dI, double* acc, float* loss, hipStream_t s) {
  int grid = (int)((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_loss, dim3(grid), dim3(256), 0, s, I, T, n, dI, acc);
  hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(1), 0, s, acc, n, loss);
  return hipGetLastError();
}
hipError_t launch_hf_tris(const DevScene& sc, Tri* tris, const float* h, float* hb, hipStream_t s) {
  int nhf = 2 * (sc.hf_G - 1) * (sc.hf_G - 1);
  hipLaunchKernelGGL(k_hf_tris, dim3((nhf + 255) / 256), dim3(256), 0, s, sc, tris, h);
  hipLaunchKernelGGL(k_hf_bounds, dim3(1), dim3(1024), 0, s, h, sc.hf_G * sc.hf_G, hb);
  return hipGetLastError();
}

}  // namespace lt
