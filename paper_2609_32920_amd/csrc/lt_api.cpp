// Host runtime and C ABI of the light tracer (see include/lt.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lt.h"
#include "lt_common.h"
#include "lt_launch.h"

using namespace lt;

namespace {

// ------------------------------------------------------------ BVH builder
// Binned SAH over triangle bounds (16 bins per axis); a node of at most 4
// triangles becomes a leaf when the SAH cost of its best split is no lower;
// median split below a depth that keeps the traversal stack within
// kStackMax.
struct BPrim { float lo[3], hi[3], c[3]; int id; };
struct BNode { float lo[3], hi[3]; int left = -1, right = -1, first = 0, count = 0; };

struct Builder {
  std::vector<BPrim> prims;
  std::vector<BNode> bn;
  int max_depth = 0;

  static void grow(float* lo, float* hi, const float* plo, const float* phi) {
    for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], plo[a]); hi[a] = std::max(hi[a], phi[a]); }
  }
  static float area(const float* lo, const float* hi) {
    float d[3];
    for (int a = 0; a < 3; ++a) d[a] = std::max(0.0f, hi[a] - lo[a]);
    return 2.0f * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
  }

  int build(int b, int e, int depth) {
    int idx = (int)bn.size();
    bn.emplace_back();
    BNode nd;
    for (int a = 0; a < 3; ++a) { nd.lo[a] = 3e38f; nd.hi[a] = -3e38f; }
    float clo[3] = {3e38f, 3e38f, 3e38f}, chi[3] = {-3e38f, -3e38f, -3e38f};
    for (int i = b; i < e; ++i) {
      grow(nd.lo, nd.hi, prims[i].lo, prims[i].hi);
      grow(clo, chi, prims[i].c, prims[i].c);
    }
    max_depth = std::max(max_depth, depth);
    int n = e - b;
    if (n <= 1) { nd.first = b; nd.count = n; bn[idx] = nd; return idx; }
    int mid = -1;
    if (depth < kStackMax - 8) {
      const int NB = 16;
      float best = 3e38f; int best_axis = -1, best_bin = -1;
      for (int a = 0; a < 3; ++a) {
        float ext = chi[a] - clo[a];
        if (!(ext > 0.0f)) continue;
        int cnt[NB] = {0};
        float blo[NB][3], bhi[NB][3];
        for (int k = 0; k < NB; ++k) for (int q = 0; q < 3; ++q) { blo[k][q] = 3e38f; bhi[k][q] = -3e38f; }
        for (int i = b; i < e; ++i) {
          int k = std::min(NB - 1, (int)((prims[i].c[a] - clo[a]) / ext * NB));
          cnt[k]++;
          grow(blo[k], bhi[k], prims[i].lo, prims[i].hi);
        }
        for (int s = 1; s < NB; ++s) {
          float llo[3] = {3e38f, 3e38f, 3e38f}, lhi[3] = {-3e38f, -3e38f, -3e38f};
          float rlo[3] = {3e38f, 3e38f, 3e38f}, rhi[3] = {-3e38f, -3e38f, -3e38f};
          int nl = 0, nr = 0;
          for (int k = 0; k < s; ++k) if (cnt[k]) { grow(llo, lhi, blo[k], bhi[k]); nl += cnt[k]; }
          for (int k = s; k < NB; ++k) if (cnt[k]) { grow(rlo, rhi, blo[k], bhi[k]); nr += cnt[k]; }
          if (!nl || !nr) continue;
          float cost = area(llo, lhi) * nl + area(rlo, rhi) * nr;
          if (cost < best) { best = cost; best_axis = a; best_bin = s; }
        }
      }
      // SAH termination: a leaf of up to 4 costs n intersection tests; a
      // split costs one node visit (two box tests) plus the area-weighted
      // tests below it
      if (n <= 4 && (best_axis < 0 || 1.0f + best / std::max(area(nd.lo, nd.hi), 1e-30f) >= (float)n)) {
        nd.first = b; nd.count = n; bn[idx] = nd; return idx;
      }
      if (best_axis >= 0) {
        float ext = chi[best_axis] - clo[best_axis];
        auto it = std::partition(prims.begin() + b, prims.begin() + e, [&](const BPrim& p) {
          int k = std::min(NB - 1, (int)((p.c[best_axis] - clo[best_axis]) / ext * NB));
          return k < best_bin;
        });
        mid = (int)(it - prims.begin());
        if (mid == b || mid == e) mid = -1;
      }
    }
    if (mid < 0) {  // object median on the widest centroid axis
      int a = 0;
      for (int q = 1; q < 3; ++q) if (chi[q] - clo[q] > chi[a] - clo[a]) a = q;
      mid = (b + e) / 2;
      std::nth_element(prims.begin() + b, prims.begin() + mid, prims.begin() + e,
                       [a](const BPrim& x, const BPrim& y) { return x.c[a] < y.c[a]; });
    }
    int l = build(b, mid, depth + 1);
    int r = build(mid, e, depth + 1);
    nd.left = l; nd.right = r;
    bn[idx] = nd;
    return idx;
  }
};

void pad_box(const float* lo, const float* hi, float* plo, float* phi) {
  for (int a = 0; a < 3; ++a) {
    float pad = 1e-5f + 1e-6f * std::max(std::fabs(lo[a]), std::fabs(hi[a]));
    plo[a] = lo[a] - pad; phi[a] = hi[a] + pad;
  }
}

struct Flat {
  std::vector<Node> nodes;
  std::vector<int> depth;
};

int flatten(const Builder& B, int bi, int depth, Flat& F) {
  int idx = (int)F.nodes.size();
  F.nodes.emplace_back();
  F.depth.push_back(depth);
  const BNode& b = B.bn[bi];
  Node nd;
  std::memset(&nd, 0, sizeof(nd));
  int kids[2] = {b.left, b.right};
  int cidx[2], ccnt[2];
  float lo[2][3], hi[2][3];
  for (int k = 0; k < 2; ++k) {
    const BNode& c = B.bn[kids[k]];
    pad_box(c.lo, c.hi, lo[k], hi[k]);
    if (c.left < 0) { cidx[k] = c.first; ccnt[k] = c.count; }
    else { cidx[k] = flatten(B, kids[k], depth + 1, F); ccnt[k] = 0; }
  }
  for (int a = 0; a < 3; ++a) {
    nd.lo0[a] = lo[0][a]; nd.hi0[a] = hi[0][a];
    nd.lo1[a] = lo[1][a]; nd.hi1[a] = hi[1][a];
  }
  nd.child0 = cidx[0]; nd.child1 = cidx[1]; nd.count0 = ccnt[0]; nd.count1 = ccnt[1];
  F.nodes[idx] = nd;
  return idx;
}

template <typename T>
hipError_t upload(T** dst, const T* src, size_t n) {
  if (*dst) { hipFree(*dst); *dst = nullptr; }
  if (n == 0) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

// Device scratch of the no-allocation entry point (lt_backward_lrb3_noalloc):
// work counters and statistics, the FP64 emitter-gradient accumulators and
// the LRB-3 hand-off.  One copy per GPU, held from module load to process
// end; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (the array's name is a host-side stand-in).
constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr size_t kScratchCounters = 0, kScratchAcc = kCtrBytes, kScratchHand = kCtrBytes + 256;
static __device__ __align__(256) char scratch[kScratchBytes];

struct lt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  lt_tuning tune{128, 10, 1, 2};
  uint64_t cap = 0;
  lt_stats stats{};
  int n_cu = 256;
  int lds_max = 65536;  // dynamic LDS bytes one workgroup may use
  bool has_scene = false;
  Node* d_nodes = nullptr;
  Tri* d_tris = nullptr;
  int32_t* d_prim_mat = nullptr;
  float* d_prim_uv = nullptr;
  int32_t* d_mat_type = nullptr;
  int32_t* d_mat_tex = nullptr;
  float* d_mat_ior = nullptr;
  float* d_hfb = nullptr;          // least and greatest height [2]
  DevScene dsc{};
  size_t scene_bytes = 0;
  unsigned int* d_counter = nullptr;
  double* d_acc = nullptr;  // [0..2] emitter gradient, [3] loss
  bool guide_ok = false;     // guide kernels got the LDS they need
  void* d_gpack = nullptr;   // packed bf16 guide operands
  float4* d_grec = nullptr;  // guided emission records [grec_n]
  size_t grec_n = 0;
  float* d_gpart = nullptr;  // guide gradient partial sums [gpart_n][kGN + 1]
  size_t gpart_n = 0;
  float* d_tcx = nullptr;    // albedo texel centres [n_texels][3] (diffuse guide inputs)
  float* d_tcn = nullptr;    // and their normals (0: no triangle covers the centre)
  float4* d_gtab = nullptr;  // diffuse guide table [2 n_texels][16], built per guided pass
  char* d_hand = nullptr;    // LRB-3 hand-off between its two kernels [hand_n bytes]
  size_t hand_n = 0;
  char* d_scratch = nullptr; // this device's copy of the static scratch (null: unavailable)
  bool has_conductor = false; // the uploaded scene has rough-conductor surfaces
  bool hf_lambert = false;    // the heightfield is Lambertian

  lt_status fail(lt_status s, const char* fmt, const char* a = "") {
    char buf[512];
    std::snprintf(buf, sizeof(buf), fmt, a);
    err = buf;
    return s;
  }
  lt_status hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return LT_OK;
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
    err = buf;
    return LT_ERR_HIP;
  }
  void free_scene() {
    hipFree(d_nodes); hipFree(d_tris); hipFree(d_prim_mat); hipFree(d_prim_uv);
    hipFree(d_mat_type); hipFree(d_mat_tex); hipFree(d_mat_ior); hipFree(d_hfb);
    hipFree(d_tcx); hipFree(d_tcn); hipFree(d_gtab);
    d_nodes = nullptr; d_tris = nullptr; d_prim_mat = nullptr; d_prim_uv = nullptr; d_mat_type = nullptr;
    d_mat_tex = nullptr; d_mat_ior = nullptr; d_hfb = nullptr;
    d_tcx = nullptr; d_tcn = nullptr; d_gtab = nullptr;
    has_scene = false; scene_bytes = 0;
  }
};

namespace {

int persistent_grid(const lt_ctx* c, int64_t n, int block) {
  int64_t g = (int64_t)c->n_cu * c->tune.blocks_per_cu;
  int64_t need = (n + block - 1) / block;
  return (int)std::max<int64_t>(1, std::min(g, need));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Heights gradients go to a per-workgroup LDS copy when it fits next to the
// traversal stacks of a `block`-thread workgroup.  The replay kernels (arithmetic-
// heavy, latency-bound at two or three waves per SIMD) take it only when it
// costs no resident workgroups per CU; the tape walk (little arithmetic per
// scatter, bound by the atomics) takes it whenever it fits.
int hgrad_in_lds(const lt_ctx* c, const float* g_heights, BwdKernel k, int block, size_t stack, bool keep_residency) {
  if (!g_heights || c->dsc.hf_G < 2) return 0;
  size_t need = (size_t)c->dsc.hf_G * c->dsc.hf_G * sizeof(float);
  if (stack + need > (size_t)c->lds_max) return 0;
  if (!keep_residency) return 1;
  int with = resident_groups(k, block, stack + need);
  return with > 0 && with >= resident_groups(k, block, stack) ? 1 : 0;
}

// Workgroup size of the attached replay backwards.  The LRB-3 kernel holds
// three waves per SIMD and the ResLRB kernel two, so one workgroup of `big`
// threads (768, 512) fills a CU and has the CU's whole LDS: the traversal
// stacks plus a heights-gradient copy that 256-thread workgroups could not
// hold without losing residency (128² heights: caustic LRB-3 backward
// 51.1 -> 48.8 ms).  256 where the copy fits those anyway (small
// heightfields run 1-2% faster so) or does not fit beside `big` lanes'
// stacks either.
int att_replay_block(const lt_ctx* c, const float* g_heights, int stack_n, BwdKernel k, int big) {
  if (!g_heights || c->dsc.hf_G < 2) return 256;
  const size_t need = (size_t)c->dsc.hf_G * c->dsc.hf_G * sizeof(float);
  auto copy_free = [&](int block) {
    const size_t stack = (size_t)stack_n * block * sizeof(int);
    if (stack + need > (size_t)c->lds_max) return false;
    int with = resident_groups(k, block, stack + need);
    return with > 0 && with >= resident_groups(k, block, stack);
  };
  return !copy_free(256) && copy_free(big) ? big : 256;
}

// Albedo gradients go to a per-workgroup LDS copy (lt_tuning.lds_grad) when
// the texture set takes at most 48 KB, fits next to the other LDS users and
// costs the kernel no resident workgroups per CU; otherwise each wave
// write-combines them into the caller's array.
int agrad_in_lds(const lt_ctx* c, BwdKernel k, int block, size_t used) {
  if (!c->tune.lds_grad) return 0;
  size_t need = (size_t)c->dsc.n_tex * c->dsc.tex_res * c->dsc.tex_res * 3 * sizeof(float);
  if (need > 48 * 1024 || used + need > (size_t)c->lds_max) return 0;
  int with = resident_groups(k, block, used + need);
  return with > 0 && with >= resident_groups(k, block, used) ? 1 : 0;
}
size_t stack_lds(const lt_ctx* c, int block) { return (size_t)c->dsc.stack_n * block * sizeof(int); }
size_t agrad_lds_bytes(const lt_ctx* c, int on) {
  return on ? (size_t)c->dsc.n_tex * c->dsc.tex_res * c->dsc.tex_res * 3 * sizeof(float) : 0;
}
// Textured-emitter gradients go to a per-workgroup LDS copy (after the
// albedo copy; `used` bytes before it) when lds_grad allows copies, the
// texture takes at most 16 KB and the copy costs the kernel no resident
// workgroups; otherwise each path adds to the caller's array.
int legrad_in_lds(const lt_ctx* c, BwdKernel k, int block, size_t used) {
  if (!c->tune.lds_grad || c->dsc.em_tex_res <= 0) return 0;
  const size_t need = (size_t)c->dsc.em_tex_res * c->dsc.em_tex_res * 3 * sizeof(float);
  if (need > 16 * 1024 || used + need > (size_t)c->lds_max) return 0;
  const int with = resident_groups(k, block, used + need);
  return with > 0 && with >= resident_groups(k, block, used) ? 1 : 0;
}

// Launch shape of a detached replay backward.  An LDS copy of the albedo
// gradients is held per workgroup, so at the tuned shape (128 threads, ten
// workgroups per CU) it would cost resident workgroups and is left out; the
// same threads per CU in fewer, larger workgroups hold fewer copies.  The
// first of block, 2 block, 4 block ... (at most 1024 threads, while the
// workgroups per CU divide evenly) at which the copy fits without a loss of
// residency is taken (256x256 box, fused LRB-3 backward: 6.83 -> 6.31 ms),
// the tuned shape when there is none.
// stack_n: traversal stack entries per lane (a batch's common depth, else
// the scene's)
struct Shape { int block, grid, agrad_lds; };
Shape replay_shape(const lt_ctx* c, BwdKernel k, int64_t n, int stack_n) {
  const int b0 = c->tune.block, k0 = c->tune.blocks_per_cu;
  for (int f = 1; b0 * f <= 1024 && k0 % f == 0; f *= 2) {
    const int blk = b0 * f;
    if (!agrad_in_lds(c, k, blk, (size_t)stack_n * blk * sizeof(int))) continue;
    const int64_t g = (int64_t)c->n_cu * (k0 / f), need = (n + blk - 1) / blk;
    return {blk, (int)std::max<int64_t>(1, std::min(g, need)), 1};
  }
  return {b0, persistent_grid(c, n, b0), 0};
}
Shape replay_shape(const lt_ctx* c, BwdKernel k, int64_t n) { return replay_shape(c, k, n, c->dsc.stack_n); }
size_t hgrad_lds_bytes(const lt_ctx* c, int on) { return on ? (size_t)c->dsc.hf_G * c->dsc.hf_G * sizeof(float) : 0; }

struct SideLayout { size_t tape = 0, len = 0, emit = 0, gw = 0, res = 0, spl_hdr = 0, spl = 0, total = 0; };

// Side state: naive tape [D][N] records (+ N path lengths; attached: + the
// emitted ray's dv_1/dH_1 per path; detached with a diffuse guide or rough
// conductors in the scene: + [D][N] scatter weights), ResLRB records [N].
SideLayout side_layout(const lt_ctx* c, const lt_trace_args* a) {
  SideLayout L;
  size_t N = (size_t)a->n_paths, D = (size_t)a->max_depth;
  const bool att = (a->flags & LT_ATTACHED) != 0;
  size_t off = 0;
  if (a->flags & LT_RECORD_TAPE) {
    L.tape = off; off = align256(off + N * D * (att ? sizeof(TapeRecAtt) : sizeof(TapeRec)));
    L.len = off; off = align256(off + N * sizeof(int32_t));
    if (att) { L.emit = off; off = align256(off + N * 2 * sizeof(float)); }
    // detached tape with a diffuse guide or rough conductors: the scatter
    // weight over rho of every vertex (the attached record has room for it)
    if (!att && ((a->flags & LT_GUIDE_DIFFUSE) || (c && c->has_conductor))) {
      L.gw = off; off = align256(off + N * D * sizeof(float));
    }
  }
  if (a->flags & LT_RECORD_RESERVOIR) {
    L.res = off; off = align256(off + N * (att ? sizeof(ResRecAtt) : sizeof(ResRec)));
  }
  if (a->flags & LT_RECORD_SPLATS) {
    L.spl_hdr = off; off = align256(off + N * sizeof(SplatHdr));
    L.spl = off; off = align256(off + N * D * sizeof(SplatRec));
  }
  L.total = off;
  return L;
}

lt_status check_args(lt_ctx* c, const lt_trace_args* a, const lt_params* p) {
  if (!c) return LT_ERR_ARG;
  if (!a || !p) return c->fail(LT_ERR_ARG, "null args or params%s");
  if (!c->has_scene) return c->fail(LT_ERR_STATE, "no scene uploaded%s");
  if (a->n_paths < 1 || a->n_paths >= (int64_t)1 << 31) return c->fail(LT_ERR_ARG, "n_paths out of range [1, 2^31)%s");
  if (a->max_depth < 1 || a->max_depth > kMaxDepth) return c->fail(LT_ERR_ARG, "max_depth out of range [1, 64]%s");
  if (a->flags & ~(uint32_t)(LT_ATTACHED | LT_SPLAT_SELECTED | LT_RECORD_TAPE | LT_RECORD_RESERVOIR | LT_CONTRIB_ADJOINT |
                             LT_RECORD_SPLATS | LT_GUIDE_DIFFUSE))
    return c->fail(LT_ERR_ARG, "unknown flag bits%s");
  if ((a->flags & LT_GUIDE_DIFFUSE) && !p->guide_w)
    return c->fail(LT_ERR_ARG, "LT_GUIDE_DIFFUSE needs params->guide_w%s");
  if ((a->flags & LT_RECORD_SPLATS) && (a->flags & (LT_ATTACHED | LT_RECORD_TAPE)))
    return c->fail(LT_ERR_UNSUPPORTED, "LT_RECORD_SPLATS is detached and not combined with LT_RECORD_TAPE%s");
  if (!p->albedo || !p->emitter_L) return c->fail(LT_ERR_ARG, "albedo and emitter_L are required%s");
  if ((a->flags & LT_ATTACHED) && c->dsc.hf_G < 2) return c->fail(LT_ERR_ARG, "LT_ATTACHED needs a heightfield%s");
  if ((a->flags & LT_ATTACHED) && c->hf_lambert)
    return c->fail(LT_ERR_UNSUPPORTED,
                   "LT_ATTACHED differentiates dielectric and rough-conductor heightfields; a Lambertian one is "
                   "detached only%s");
  if ((a->flags & LT_ATTACHED) && !p->heights) return c->fail(LT_ERR_ARG, "LT_ATTACHED needs params->heights%s");
  if (p->normal_map && (c->dsc.hf_G < 2 || !p->heights))
    return c->fail(LT_ERR_ARG, "a normal map needs a heightfield and params->heights%s");
  if (p->guide_w && c->dsc.em_type != LT_EMIT_QUAD) return c->fail(LT_ERR_UNSUPPORTED, "the emission guide needs an area emitter%s");
  if (c->dsc.em_tex_res > 0 && (a->flags & LT_ATTACHED))
    return c->fail(LT_ERR_UNSUPPORTED, "a textured emitter is supported by detached passes only%s");
  if (c->dsc.em_tex_res > 0 && p->guide_w)
    return c->fail(LT_ERR_UNSUPPORTED, "the emission guide takes an untextured emitter%s");
  if (p->guide_w && !c->guide_ok) return c->fail(LT_ERR_UNSUPPORTED, "guide kernels could not get their LDS%s");
  return LT_OK;
}

size_t guide_bytes(const lt_trace_args* a, const lt_params* p) {
  return p && p->guide_w ? (size_t)a->n_paths * sizeof(float4) : 0;
}

// LRB-3 hand-off between the pass-2 and pass-3 kernels: one entry per path
// at most (flat in depth).
// Whether lt_backward_lrb3 runs its passes as two kernels for these args
// (default 2: attached only).  On the 128x128 caustic (attached) the split
// pair runs 15.9 against 23.1 ms fused; detached the two run alike on the
// 256x256 box at depth 32 (6.28 against 6.24 ms) and the pair gains 11% on
// the glass slab (1.67 against 1.88 ms) for 40 bytes of hand-off per path,
// where the fused kernel needs none, so the detached backward stays fused
// unless asked.
bool lrb3_split(const lt_ctx* c, const lt_trace_args* a) {
  return c->tune.lrb3_split == 1 || (c->tune.lrb3_split == 2 && (a->flags & LT_ATTACHED));
}
// entries per class region of the hand-off: ceil(n_paths / 8)
uint32_t hand_region(int64_t n_paths) { return (uint32_t)((n_paths + kWorkClasses - 1) / kWorkClasses); }
size_t hand_bytes(const lt_ctx* c, const lt_trace_args* a) {
  if (!lrb3_split(c, a) || a->n_paths < 1) return 0;
  return (size_t)kWorkClasses * hand_region(a->n_paths) *
         ((a->flags & LT_ATTACHED) ? sizeof(Lrb3HandAtt) : sizeof(Lrb3Hand));
}

template <typename T>
lt_status grow(lt_ctx* c, T** ptr, size_t& have, size_t need, const char* what) {
  if (have >= need && *ptr) return LT_OK;
  hipFree(*ptr);
  *ptr = nullptr; have = 0;
  if (hipMalloc((void**)ptr, need * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return c->fail(LT_ERR_OOM, "out of device memory for %s", what);
  }
  have = need;
  return LT_OK;
}

lt_status guide_pack(lt_ctx* c, const float* w) {
  if (!c->d_gpack && hipMalloc(&c->d_gpack, guide_packed_bytes()) != hipSuccess) {
    (void)hipGetLastError();
    c->d_gpack = nullptr;
    return c->fail(LT_ERR_OOM, "out of device memory for the guide weights%s");
  }
  return c->hip(launch_guide_pack(w, c->d_gpack, c->stream), "guide pack");
}

int guide_grid(const lt_ctx* c, int64_t count) {
  int64_t blocks = ((count + 63) / 64 + 3) / 4;
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, (int64_t)c->n_cu * 4));
}

GuideArgs guide_args(lt_ctx* c, const float* w, int64_t count) {
  GuideArgs G;
  std::memset(&G, 0, sizeof(G));
  G.sc = c->dsc;
  G.count = count;
  G.w = w;
  G.packed = (const lt_u32x4*)c->d_gpack;
  return G;
}

// Guided passes: the direction and density of every path's emission, drawn
// once per pass by the guide kernel and read by the tracing kernels.
lt_status guide_prepass(lt_ctx* c, const lt_trace_args* a, const lt_params* p, PassArgs& A) {
  A.guide_rec = nullptr;
  if (!p->guide_w) return LT_OK;
  lt_status st = grow(c, &c->d_grec, c->grec_n, (size_t)a->n_paths, "guided emission records");
  if (st != LT_OK) return st;
  if ((st = guide_pack(c, p->guide_w)) != LT_OK) return st;
  GuideArgs G = guide_args(c, p->guide_w, a->n_paths);
  G.seed = a->seed;
  G.rec = c->d_grec;
  if ((st = c->hip(launch_guide_emit(G, guide_grid(c, a->n_paths), c->stream), "guide emit")) != LT_OK) return st;
  A.guide_rec = c->d_grec;
  A.gtab = nullptr;
  if (a->flags & LT_GUIDE_DIFFUSE) {
    const int64_t ne = 2 * (int64_t)c->dsc.n_tex * c->dsc.tex_res * c->dsc.tex_res;
    if (!c->d_gtab && hipMalloc((void**)&c->d_gtab, (size_t)ne * kGTabF4 * sizeof(float4)) != hipSuccess) {
      (void)hipGetLastError();
      c->d_gtab = nullptr;
      return c->fail(LT_ERR_OOM, "out of device memory for the diffuse guide table%s");
    }
    GuideArgs T = guide_args(c, p->guide_w, ne);
    T.x = c->d_tcx; T.n = c->d_tcn; T.table = c->d_gtab;
    if ((st = c->hip(launch_guide_table(T, guide_grid(c, ne), c->stream), "guide table")) != LT_OK) return st;
    A.gtab = c->d_gtab;
  }
  return LT_OK;
}

// The heightfield's triangles and height bounds from params->heights (the
// BVH holds the static triangles only, so nothing else changes with them).
lt_status prepare_geometry(lt_ctx* c, const lt_params* p) {
  if (c->dsc.hf_G < 2 || !p->heights) return LT_OK;
  return c->hip(launch_hf_tris(c->dsc, c->d_tris, p->heights, c->d_hfb, c->stream), "hf tris");
}

PassArgs base_args(lt_ctx* c, const lt_trace_args* a, const lt_params* p) {
  PassArgs A;
  std::memset(&A, 0, sizeof(A));
  A.sc = c->dsc;
  A.seed = a->seed;
  A.n_paths = (int32_t)a->n_paths;
  A.D = a->max_depth;
  A.flags = a->flags;
  double Kfilm = (double)c->dsc.W * c->dsc.H / ((double)c->dsc.film_area * (double)a->n_paths);
  A.Kfilm = (float)Kfilm;
  A.n_texels = c->dsc.n_tex * c->dsc.tex_res * c->dsc.tex_res;
  A.hgrad_lds = 0;
  A.agrad_lds = 0;
  A.mask = a->path_mask;
  A.sig = a->path_sig;
  A.info = a->path_info;
  A.albedo = p->albedo;
  A.Le = p->emitter_L;
  A.heights = p->heights;
  A.nmap = p->normal_map;
  A.cond = c->has_conductor ? 1 : 0;
  A.counter = c->d_counter;
  A.stats = reinterpret_cast<unsigned long long*>(c->d_counter + kCtrStats);  // same allocation
  return A;
}

lt_status check_cap(lt_ctx* c, size_t side) {
  if (c->cap && side + c->scene_bytes + 64 > c->cap) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "memory cap exceeded: %zu side-state bytes + %zu library bytes > %llu",
                  side, c->scene_bytes + 64, (unsigned long long)c->cap);
    c->err = buf;
    return LT_ERR_OOM;
  }
  return LT_OK;
}

}  // namespace

extern "C" {

lt_status lt_create(int device, void* stream, lt_ctx** out) {
  if (!out) return LT_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LT_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return LT_ERR_HIP;
  lt_ctx* c = new (std::nothrow) lt_ctx();
  if (!c) return LT_ERR_OOM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    c->lds_max = lds;
  if (set_lds_limit(c->lds_max) != hipSuccess) {
    (void)hipGetLastError();
    c->lds_max = 65536;
  }
  c->guide_ok = guide_init() == hipSuccess;
  if (!c->guide_ok) (void)hipGetLastError();
  if (hipMalloc((void**)&c->d_counter, kCtrBytes) != hipSuccess || hipMalloc((void**)&c->d_acc, 256) != hipSuccess) {
    hipFree(c->d_counter); hipFree(c->d_acc);
    delete c;
    return LT_ERR_OOM;
  }
  // the static scratch's address on this device (the device is current)
  void* sp = nullptr;
  if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) == hipSuccess && sp) {
    c->d_scratch = static_cast<char*>(sp);
  } else {
    (void)hipGetLastError();
    c->d_scratch = nullptr;
  }
  *out = c;
  return LT_OK;
}

void lt_destroy(lt_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  c->free_scene();
  hipFree(c->d_counter);
  hipFree(c->d_acc);
  hipFree(c->d_gpack);
  hipFree(c->d_grec);
  hipFree(c->d_gpart);
  hipFree(c->d_hand);
  delete c;
}

const char* lt_last_error(const lt_ctx* c) { return c ? c->err.c_str() : "null context"; }

lt_status lt_set_stream(lt_ctx* c, void* stream) {
  if (!c) return LT_ERR_ARG;
  c->stream = (hipStream_t)stream;
  return LT_OK;
}

lt_status lt_set_tuning(lt_ctx* c, const lt_tuning* t) {
  if (!c) return LT_ERR_ARG;
  if (!t) { c->tune = lt_tuning{128, 10, 1, 2}; return LT_OK; }
  if (t->block < 64 || t->block > 1024 || (t->block % 64) != 0) return c->fail(LT_ERR_ARG, "block must be 64..1024, a multiple of 64%s");
  if (t->blocks_per_cu < 1 || t->blocks_per_cu > 64) return c->fail(LT_ERR_ARG, "blocks_per_cu must be 1..64%s");
  if ((size_t)kStackMax * t->block * sizeof(int) > (size_t)c->lds_max) return c->fail(LT_ERR_ARG, "traversal stack exceeds the LDS of a workgroup%s");
  if (t->lds_grad != 0 && t->lds_grad != 1) return c->fail(LT_ERR_ARG, "lds_grad must be 0 or 1%s");
  if (t->lrb3_split < 0 || t->lrb3_split > 2) return c->fail(LT_ERR_ARG, "lrb3_split must be 0, 1 or 2%s");
  c->tune = *t;
  return LT_OK;
}

lt_status lt_get_tuning(const lt_ctx* c, lt_tuning* out) {
  if (!c || !out) return LT_ERR_ARG;
  *out = c->tune;
  return LT_OK;
}

lt_status lt_set_memory_cap(lt_ctx* c, uint64_t bytes) {
  if (!c) return LT_ERR_ARG;
  c->cap = bytes;
  return LT_OK;
}

lt_status lt_get_stats(const lt_ctx* c, lt_stats* out) {
  if (!c || !out) return LT_ERR_ARG;
  uint64_t s[2] = {0, 0};
  if (hipStreamSynchronize(c->stream) != hipSuccess ||
      hipMemcpy(s, c->d_counter + kCtrStats, sizeof(s), hipMemcpyDeviceToHost) != hipSuccess)
    return LT_ERR_HIP;
  out->guard_triggers = s[0];
  out->nonfinite = s[1];
  return LT_OK;
}

lt_status lt_read_counters(lt_ctx* c, uint64_t* out16, int reset) {
  if (!c || !out16) return LT_ERR_ARG;
  hipError_t e = read_counters(out16, reset != 0, c->stream);
  if (e == hipErrorNotSupported) return c->fail(LT_ERR_UNSUPPORTED, "library built without LT_COUNTERS%s");
  return c->hip(e, "read counters");
}

lt_status lt_scene_upload(lt_ctx* c, const lt_scene_desc* s) {
  if (!c) return LT_ERR_ARG;
  if (!s) return c->fail(LT_ERR_ARG, "null scene%s");
  if (s->n_tris < 0 || (s->n_tris > 0 && (!s->tri_v || !s->tri_uv || !s->tri_mat)))
    return c->fail(LT_ERR_ARG, "bad triangle arrays%s");
  if (s->n_mats < 1 || !s->mat_type || !s->mat_tex || !s->mat_ior) return c->fail(LT_ERR_ARG, "bad material arrays%s");
  if (s->n_tex < 1 || s->tex_res < 1 || (int64_t)s->n_tex * s->tex_res * s->tex_res >= (1 << 27))
    return c->fail(LT_ERR_ARG, "bad texture shape%s");
  if (s->width < 1 || s->height < 1 || s->width > 16384 || s->height > 16384) return c->fail(LT_ERR_ARG, "bad film size%s");
  if (!(s->cam_fov_deg > 0.0 && s->cam_fov_deg < 180.0)) return c->fail(LT_ERR_ARG, "bad field of view%s");
  if (s->em_type != LT_EMIT_QUAD && s->em_type != LT_EMIT_POINT && s->em_type != LT_EMIT_DIRECTIONAL)
    return c->fail(LT_ERR_ARG, "bad emitter type%s");
  if (s->em_tex_res < 0 || s->em_tex_res > 4096 || (s->em_tex_res > 0 && s->em_type == LT_EMIT_POINT))
    return c->fail(LT_ERR_ARG, "bad emitter texture size (0, or 1..4096 on a quad or directional emitter)%s");
  if (s->hf_G == 1 || s->hf_G < 0 || s->hf_G > 4096) return c->fail(LT_ERR_ARG, "bad heightfield size%s");
  for (int m = 0; m < s->n_mats; ++m) {
    if (s->mat_type[m] < 0 || s->mat_type[m] > 3) return c->fail(LT_ERR_ARG, "bad material type%s");
    if ((s->mat_type[m] == LT_MAT_LAMBERT || s->mat_type[m] == LT_MAT_CONDUCTOR) &&
        (s->mat_tex[m] < 0 || s->mat_tex[m] >= s->n_tex))
      return c->fail(LT_ERR_ARG, "Lambertian or conductor material without a valid texture%s");
    if (s->mat_type[m] == LT_MAT_CONDUCTOR && !(s->mat_ior[m] >= 1e-3 && s->mat_ior[m] <= 1.0))
      return c->fail(LT_ERR_ARG, "conductor roughness outside [1e-3, 1]%s");
    if (s->mat_type[m] == LT_MAT_DIELECTRIC && !(s->mat_ior[m] > 0.0)) return c->fail(LT_ERR_ARG, "bad IOR%s");
  }
  for (int t = 0; t < s->n_tris; ++t)
    if (s->tri_mat[t] < 0 || s->tri_mat[t] >= s->n_mats) return c->fail(LT_ERR_ARG, "triangle material out of range%s");
  if (s->hf_G >= 2 && (s->hf_mat < 0 || s->hf_mat >= s->n_mats)) return c->fail(LT_ERR_ARG, "heightfield material out of range%s");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(LT_ERR_HIP, "hipSetDevice failed%s");

  const int G = s->hf_G;
  const int n_static = s->n_tris;
  const int n_hf = G >= 2 ? 2 * (G - 1) * (G - 1) : 0;
  const int n_prims = n_static + n_hf;
  if (n_prims < 1) return c->fail(LT_ERR_ARG, "scene has no geometry%s");

  // primitive geometry (double -> float), heightfield flat (h = 0)
  std::vector<Tri> tri(n_prims);
  auto setv = [](Tri& t, const double* v0, const double* v1, const double* v2, int prim) {
    for (int a = 0; a < 3; ++a) {
      t.p0[a] = (float)v0[a];
      t.e1[a] = (float)(v1[a] - v0[a]);
      t.e2[a] = (float)(v2[a] - v0[a]);
    }
    t.prim = prim; t.pad1 = t.pad2 = 0.f;
  };
  for (int t = 0; t < n_static; ++t)
    setv(tri[t], s->tri_v + t * 9, s->tri_v + t * 9 + 3, s->tri_v + t * 9 + 6, t);
  for (int q = 0; q < n_hf; ++q) {
    int cell = q >> 1, half = q & 1, ci = cell % (G - 1), cj = cell / (G - 1);
    static const int o0[3][2] = {{0, 0}, {1, 1}, {1, 0}};
    static const int o1[3][2] = {{0, 0}, {0, 1}, {1, 1}};
    const int (*o)[2] = half == 0 ? o0 : o1;
    double v[3][3];
    for (int k = 0; k < 3; ++k) {
      v[k][0] = s->hf_x0 + (ci + o[k][0]) * s->hf_dx;
      v[k][1] = s->hf_base;
      v[k][2] = s->hf_z0 + (cj + o[k][1]) * s->hf_dx;
    }
    setv(tri[n_static + q], v[0], v[1], v[2], n_static + q);
  }

  // the BVH over the static triangles (the heightfield is walked as a grid)
  Builder B;
  B.prims.resize(n_static);
  for (int i = 0; i < n_static; ++i) {
    BPrim& p = B.prims[i];
    const Tri& t = tri[i];
    for (int a = 0; a < 3; ++a) {
      float v0 = t.p0[a], v1 = t.p0[a] + t.e1[a], v2 = t.p0[a] + t.e2[a];
      p.lo[a] = std::min(v0, std::min(v1, v2));
      p.hi[a] = std::max(v0, std::max(v1, v2));
      p.c[a] = 0.5f * (p.lo[a] + p.hi[a]);
    }
    p.id = i;
  }
  Flat F;
  const int root = n_static > 0 ? B.build(0, n_static, 0) : -1;
  if (root < 0) {
    // no static triangles: an empty BVH
  } else if (B.bn[root].left < 0) {  // the whole scene is one leaf
    Node nd;
    std::memset(&nd, 0, sizeof(nd));
    pad_box(B.bn[root].lo, B.bn[root].hi, nd.lo0, nd.hi0);
    for (int a = 0; a < 3; ++a) { nd.lo1[a] = 0.f; nd.hi1[a] = 0.f; }
    nd.child0 = 0; nd.count0 = B.bn[root].count; nd.child1 = -1; nd.count1 = 0;
    F.nodes.push_back(nd);
    F.depth.push_back(0);
  } else {
    flatten(B, root, 0, F);
  }
  int maxd = 0;
  for (int d : F.depth) maxd = std::max(maxd, d);
  if (maxd + 2 > kStackMax) return c->fail(LT_ERR_UNSUPPORTED, "BVH deeper than the traversal stack%s");
  // static triangles in BVH order, then the heightfield's in grid order
  std::vector<Tri> ordered(n_prims);
  for (int k = 0; k < n_static; ++k) ordered[k] = tri[B.prims[k].id];
  for (int q = 0; q < n_hf; ++q) ordered[n_static + q] = tri[n_static + q];
  std::vector<int32_t> pmat(n_prims);
  for (int t = 0; t < n_static; ++t) pmat[t] = s->tri_mat[t];
  for (int q = 0; q < n_hf; ++q) pmat[n_static + q] = s->hf_mat;
  std::vector<float> puv((size_t)std::max(n_static, 1) * 6, 0.f);
  for (int t = 0; t < n_static; ++t)
    for (int k = 0; k < 6; ++k) puv[(size_t)t * 6 + k] = (float)s->tri_uv[(size_t)t * 6 + k];
  std::vector<int32_t> mtype(s->mat_type, s->mat_type + s->n_mats), mtex(s->mat_tex, s->mat_tex + s->n_mats);
  std::vector<float> mior(s->n_mats);
  for (int m = 0; m < s->n_mats; ++m) mior[m] = (float)s->mat_ior[m];

  c->free_scene();
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(&c->d_nodes, F.nodes.data(), F.nodes.size());
  if (e == hipSuccess) e = upload(&c->d_tris, ordered.data(), ordered.size());
  if (e == hipSuccess) e = upload(&c->d_prim_mat, pmat.data(), pmat.size());
  if (e == hipSuccess) e = upload(&c->d_prim_uv, puv.data(), puv.size());
  if (e == hipSuccess) e = upload(&c->d_mat_type, mtype.data(), mtype.size());
  if (e == hipSuccess) e = upload(&c->d_mat_tex, mtex.data(), mtex.size());
  if (e == hipSuccess) e = upload(&c->d_mat_ior, mior.data(), mior.size());
  const float hb0[2] = {0.f, 0.f};  // a flat heightfield until heights arrive
  if (e == hipSuccess) e = upload(&c->d_hfb, hb0, 2);
  if (e != hipSuccess) { c->free_scene(); return c->hip(e, "scene upload"); }
  c->has_conductor = false;
  for (int t = 0; t < s->n_tris; ++t) c->has_conductor |= s->mat_type[s->tri_mat[t]] == LT_MAT_CONDUCTOR;
  if (G >= 2) c->has_conductor |= s->mat_type[s->hf_mat] == LT_MAT_CONDUCTOR;
  c->hf_lambert = G >= 2 && s->mat_type[s->hf_mat] == LT_MAT_LAMBERT;
  c->scene_bytes = F.nodes.size() * sizeof(Node) + ordered.size() * sizeof(Tri) + pmat.size() * 4 +
                   puv.size() * 4 + 8 +
                   (size_t)s->n_tex * s->tex_res * s->tex_res * 6 * sizeof(float) + 512;

  DevScene& d = c->dsc;
  std::memset(&d, 0, sizeof(d));
  d.nodes = c->d_nodes; d.tris = c->d_tris; d.prim_mat = c->d_prim_mat; d.prim_uv = c->d_prim_uv;
  d.mat_type = c->d_mat_type; d.mat_tex = c->d_mat_tex; d.mat_ior = c->d_mat_ior;
  d.n_nodes = (int)F.nodes.size(); d.n_tris = n_prims; d.n_static = n_static;
  d.hf_G = G >= 2 ? G : 0;
  d.hf_x0 = (float)s->hf_x0; d.hf_z0 = (float)s->hf_z0; d.hf_dx = (float)s->hf_dx; d.hf_base = (float)s->hf_base;
  d.hf_mat = s->hf_mat;
  d.hf_hb = c->d_hfb;
  d.n_tex = s->n_tex; d.tex_res = s->tex_res;
  d.em_type = s->em_type;
  d.em_tex_res = s->em_tex_res;
  double cr[3] = {s->em_e1[1] * s->em_e2[2] - s->em_e1[2] * s->em_e2[1],
                  s->em_e1[2] * s->em_e2[0] - s->em_e1[0] * s->em_e2[2],
                  s->em_e1[0] * s->em_e2[1] - s->em_e1[1] * s->em_e2[0]};
  double area = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  for (int a = 0; a < 3; ++a) {
    d.em_o[a] = (float)s->em_o[a]; d.em_e1[a] = (float)s->em_e1[a]; d.em_e2[a] = (float)s->em_e2[a];
    d.em_n[a] = area > 0 ? (float)(cr[a] / area) : 0.f;
  }
  d.em_area = (float)area;
  if (s->em_type != LT_EMIT_POINT && !(area > 0)) { c->free_scene(); return c->fail(LT_ERR_ARG, "degenerate quad emitter%s"); }
  {  // guide normalisation box: static triangles, heightfield footprint, emitter corners
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    auto add = [&](double x, double y, double z) {
      double p[3] = {x, y, z};
      for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], p[a]); hi[a] = std::max(hi[a], p[a]); }
    };
    for (long i = 0; i < (long)n_static * 3; ++i) add(s->tri_v[i * 3], s->tri_v[i * 3 + 1], s->tri_v[i * 3 + 2]);
    if (G >= 2) {
      double ext = (G - 1) * s->hf_dx;
      add(s->hf_x0, s->hf_base, s->hf_z0);
      add(s->hf_x0 + ext, s->hf_base, s->hf_z0 + ext);
    }
    const double *o = s->em_o, *e1 = s->em_e1, *e2 = s->em_e2;
    add(o[0], o[1], o[2]);
    if (s->em_type != LT_EMIT_POINT) {
      add(o[0] + e1[0], o[1] + e1[1], o[2] + e1[2]);
      add(o[0] + e2[0], o[1] + e2[1], o[2] + e2[2]);
      add(o[0] + e1[0] + e2[0], o[1] + e1[1] + e2[1], o[2] + e1[2] + e2[2]);
    }
    for (int a = 0; a < 3; ++a) {
      double h = 0.5 * (hi[a] - lo[a]);
      d.gb_c[a] = (float)(0.5 * (lo[a] + hi[a]));
      d.gb_ih[a] = h > 0 ? (float)(1.0 / h) : 0.f;
    }
  }
  {  // albedo texel centres for the diffuse guide table: the chart centre
     // ((tx + 1/2)/R, (ty + 1/2)/R) of each texel on the lowest-index static
     // Lambertian triangle of its texture whose chart triangle holds it
     // (barycentrics >= -1e-9); position by barycentric blend, unit normal
     // of (v1 - v0) x (v2 - v0); normal 0 where no triangle holds it
    const int R = s->tex_res;
    const size_t T = (size_t)s->n_tex * R * R;
    std::vector<float> tcx(T * 3, 0.f), tcn(T * 3, 0.f);
    std::vector<char> done(T, 0);
    for (int t = 0; t < n_static; ++t) {
      const int m = s->tri_mat[t];
      if (s->mat_type[m] != LT_MAT_LAMBERT) continue;
      const int tex = s->mat_tex[m];
      const double* uv = s->tri_uv + (size_t)t * 6;
      const double* v = s->tri_v + (size_t)t * 9;
      const double a0 = uv[2] - uv[0], a1 = uv[3] - uv[1], b0 = uv[4] - uv[0], b1 = uv[5] - uv[1];
      const double det = a0 * b1 - a1 * b0;
      if (!(std::fabs(det) > 0.0)) continue;
      double e1[3], e2[3], nr[3];
      for (int q = 0; q < 3; ++q) { e1[q] = v[3 + q] - v[q]; e2[q] = v[6 + q] - v[q]; }
      nr[0] = e1[1] * e2[2] - e1[2] * e2[1]; nr[1] = e1[2] * e2[0] - e1[0] * e2[2]; nr[2] = e1[0] * e2[1] - e1[1] * e2[0];
      const double nl = std::sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
      if (!(nl > 0.0)) continue;
      for (int ty = 0; ty < R; ++ty)
        for (int tx = 0; tx < R; ++tx) {
          const size_t k = ((size_t)tex * R + ty) * R + tx;
          if (done[k]) continue;
          const double px = (tx + 0.5) / R - uv[0], py = (ty + 0.5) / R - uv[1];
          const double w1 = (px * b1 - py * b0) / det, w2 = (a0 * py - a1 * px) / det, w0 = 1.0 - w1 - w2;
          if (w0 < -1e-9 || w1 < -1e-9 || w2 < -1e-9) continue;
          for (int q = 0; q < 3; ++q) {
            tcx[k * 3 + q] = (float)(w0 * v[q] + w1 * v[3 + q] + w2 * v[6 + q]);
            tcn[k * 3 + q] = (float)(nr[q] / nl);
          }
          done[k] = 1;
        }
    }
    hipError_t e2 = upload(&c->d_tcx, tcx.data(), tcx.size());
    if (e2 == hipSuccess) e2 = upload(&c->d_tcn, tcn.data(), tcn.size());
    if (e2 != hipSuccess) { c->free_scene(); return c->hip(e2, "texel centre upload"); }
  }
  // camera frame: f = normalize(target - pos), r = normalize(f x up), u = r x f
  double f[3], r[3], u[3];
  for (int a = 0; a < 3; ++a) f[a] = s->cam_target[a] - s->cam_pos[a];
  double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0)) { c->free_scene(); return c->fail(LT_ERR_ARG, "camera target equals position%s"); }
  for (int a = 0; a < 3; ++a) f[a] /= fl;
  const double* up = s->cam_up;
  r[0] = f[1] * up[2] - f[2] * up[1]; r[1] = f[2] * up[0] - f[0] * up[2]; r[2] = f[0] * up[1] - f[1] * up[0];
  double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(rl > 0)) { c->free_scene(); return c->fail(LT_ERR_ARG, "camera up parallel to view direction%s"); }
  for (int a = 0; a < 3; ++a) r[a] /= rl;
  u[0] = r[1] * f[2] - r[2] * f[1]; u[1] = r[2] * f[0] - r[0] * f[2]; u[2] = r[0] * f[1] - r[1] * f[0];
  for (int a = 0; a < 3; ++a) {
    d.cpos[a] = (float)s->cam_pos[a]; d.cf[a] = (float)f[a]; d.cr[a] = (float)r[a]; d.cu[a] = (float)u[a];
  }
  double th = std::tan(s->cam_fov_deg * M_PI / 360.0);
  d.tan_half = (float)th;
  d.aspect = (float)((double)s->width / (double)s->height);
  d.film_area = (float)(4.0 * ((double)s->width / s->height) * th * th);
  d.W = s->width; d.H = s->height;
  d.stack_n = maxd + 2;
  c->has_scene = true;
  c->err.clear();
  return c->hip(hipStreamSynchronize(c->stream), "scene upload sync");
}

size_t lt_side_state_bytes(const lt_ctx* c, const lt_trace_args* a) {
  if (!a || a->n_paths < 1 || a->max_depth < 1) return 0;
  return side_layout(c, a).total;
}

size_t lt_workspace_bytes(const lt_ctx* c, const lt_trace_args* a) {
  if (!c) return 0;
  size_t guide = guide_packed_bytes() + (a && a->n_paths > 0 ? (size_t)a->n_paths * sizeof(float4) : 0);
  if (a && (a->flags & LT_GUIDE_DIFFUSE))
    guide += 2 * (size_t)c->dsc.n_tex * c->dsc.tex_res * c->dsc.tex_res * kGTabF4 * sizeof(float4);
  return c->scene_bytes + 512 + guide + (a ? hand_bytes(c, a) : 0);
}

lt_status lt_trace(lt_ctx* c, const lt_trace_args* a, const lt_params* p, float* image, void* side,
                   size_t side_bytes) {
  lt_status st = check_args(c, a, p);
  if (st != LT_OK) return st;
  if (!image) return c->fail(LT_ERR_ARG, "null image%s");
  const bool att_rec = (a->flags & LT_ATTACHED) && (a->flags & (LT_RECORD_TAPE | LT_RECORD_RESERVOIR));
  if (att_rec && a->path_sig)
    return c->fail(LT_ERR_UNSUPPORTED, "path signatures come from the detached forward (no attached records)%s");
  SideLayout L = side_layout(c, a);
  if (L.total && (!side || side_bytes < L.total)) return c->fail(LT_ERR_ARG, "side state buffer too small%s");
  if ((st = check_cap(c, L.total + guide_bytes(a, p))) != LT_OK) return st;
  if ((st = prepare_geometry(c, p)) != LT_OK) return st;
  PassArgs A = base_args(c, a, p);
  A.image = image;
  A.contrib = a->path_contrib;
  if ((st = guide_prepass(c, a, p, A)) != LT_OK) return st;
  char* sb = (char*)side;
  if (att_rec) {
    if (a->flags & LT_RECORD_TAPE) {
      A.tape_att = (TapeRecAtt*)(sb + L.tape);
      A.tape_len = (int32_t*)(sb + L.len);
      A.emit_d = (float*)(sb + L.emit);
    }
    if (a->flags & LT_RECORD_RESERVOIR) A.res_att = (ResRecAtt*)(sb + L.res);
  } else {
    if (a->flags & LT_RECORD_TAPE) {
      A.tape = (TapeRec*)(sb + L.tape); A.tape_len = (int32_t*)(sb + L.len);
      if (L.gw) A.tape_gw = (float*)(sb + L.gw);
    }
    if (a->flags & LT_RECORD_RESERVOIR) A.res = (ResRec*)(sb + L.res);
    if (a->flags & LT_RECORD_SPLATS) { A.spl_hdr = (SplatHdr*)(sb + L.spl_hdr); A.spl = (SplatRec*)(sb + L.spl); }
  }
  size_t npix = (size_t)c->dsc.W * c->dsc.H * 3;
  if ((st = c->hip(launch_fill_f32(image, npix, 0.f, c->stream), "image clear")) != LT_OK) return st;
  if ((st = c->hip(launch_fill_u32(c->d_counter, kCtrBlock, 0u, c->stream), "counter clear")) != LT_OK) return st;
  if ((st = c->hip(launch_fill_u32(c->d_counter + kCtrStats, 4, 0u, c->stream), "stats clear")) != LT_OK) return st;
  bool tape = (a->flags & LT_RECORD_TAPE) != 0;
  if (att_rec) {
    bool rec = (a->flags & LT_RECORD_RESERVOIR) != 0;
    int grid = persistent_grid(c, a->n_paths, 256);
    return c->hip(launch_trace_att(A, tape, rec, grid, c->stream), "attached trace launch");
  }
  // the decision signature includes the reservoir choice R
  bool resv = (a->flags & (LT_RECORD_RESERVOIR | LT_SPLAT_SELECTED)) != 0 || a->path_sig != nullptr;
  int grid = persistent_grid(c, a->n_paths, c->tune.block);
  if (a->flags & LT_RECORD_SPLATS)
    return c->hip(launch_trace_splats(A, resv, grid, c->tune.block, c->stream), "trace launch");
  return c->hip(launch_trace(A, tape, resv, grid, c->tune.block, c->stream), "trace launch");
}

lt_status lt_loss_l2(lt_ctx* c, const float* image, const float* target, int64_t n, float* d_image, float* loss) {
  if (!c) return LT_ERR_ARG;
  if (!image || !target || !d_image || !loss || n < 1) return c->fail(LT_ERR_ARG, "bad loss arguments%s");
  lt_status st = c->hip(launch_fill_f64(c->d_acc + 3, 1, 0.0, c->stream), "loss clear");
  if (st != LT_OK) return st;
  return c->hip(launch_loss(image, target, (size_t)n, d_image, c->d_acc + 3, loss, c->stream), "loss launch");
}

// Where a backward call keeps its working memory: the counter area (the
// pass's eight work counters, LRB-3 pass 3's eight, pass 2's eight append
// counters, the two u64 statistics; lt_common.h), the FP64 emitter-gradient
// accumulators and the LRB-3 hand-off.
// The ordinary entry points use the context's buffers and grow the hand-off
// on demand; the no-allocation entry point points all three into the static
// scratch.
struct Work {
  unsigned int* counter;
  double* acc;
  char* hand;       // null: the context's hand-off, grown as needed
  size_t hand_cap;  // bytes at hand when it is set
};
Work ctx_work(lt_ctx* c) { return Work{c->d_counter, c->d_acc, nullptr, 0}; }

static lt_status backward_common(lt_ctx* c, const lt_trace_args* a, const lt_params* p, const float* d_image,
                                 lt_grads* g, PassArgs& A, size_t side, const Work& w) {
  lt_status st = check_args(c, a, p);
  if (st != LT_OK) return st;
  if (!d_image || !g) return c->fail(LT_ERR_ARG, "null d_image or grads%s");
  if (!g->albedo) return c->fail(LT_ERR_ARG, "grads->albedo is required%s");
  if ((st = check_cap(c, side + guide_bytes(a, p))) != LT_OK) return st;
  if ((st = prepare_geometry(c, p)) != LT_OK) return st;
  A = base_args(c, a, p);
  A.counter = w.counter;
  A.stats = reinterpret_cast<unsigned long long*>(w.counter + kCtrStats);
  if ((st = guide_prepass(c, a, p, A)) != LT_OK) return st;
  A.dI = d_image;
  A.g_albedo = g->albedo;
  A.g_Le_acc = w.acc;
  A.g_le_tex = c->dsc.em_tex_res > 0 ? g->emitter_L : nullptr;
  A.g_heights = g->heights;
  A.g_nmap = (a->flags & LT_ATTACHED) ? g->normal_map : nullptr;
  if ((st = c->hip(launch_fill_f64(w.acc, 3, 0.0, c->stream), "acc clear")) != LT_OK) return st;
  if ((st = c->hip(launch_fill_u32(w.counter + kCtrStats, 4, 0u, c->stream), "stats clear")) != LT_OK) return st;
  return c->hip(launch_fill_u32(w.counter, kCtrBlock, 0u, c->stream), "counter clear");
}
static lt_status backward_common(lt_ctx* c, const lt_trace_args* a, const lt_params* p, const float* d_image,
                                 lt_grads* g, PassArgs& A, size_t side) {
  return backward_common(c, a, p, d_image, g, A, side, ctx_work(c));
}

lt_status lt_backward_naive(lt_ctx* c, const lt_trace_args* a, const lt_params* p, const float* d_image,
                            const void* tape, size_t tape_bytes, lt_grads* g) {
  if (!c) return LT_ERR_ARG;
  if (a && !(a->flags & LT_RECORD_TAPE)) return c->fail(LT_ERR_ARG, "naive backward needs LT_RECORD_TAPE args%s");
  if (a && (!tape || tape_bytes < side_layout(c, a).total)) return c->fail(LT_ERR_ARG, "tape buffer too small%s");
  PassArgs A;
  lt_status st = backward_common(c, a, p, d_image, g, A, a ? side_layout(c, a).total : 0);
  if (st != LT_OK) return st;
  SideLayout L = side_layout(c, a);
  const char* sb = (const char*)tape;
  A.contrib = a->path_contrib;
  A.tape_in = (const TapeRec*)(sb + L.tape);
  A.tape_len_in = (const int32_t*)(sb + L.len);
  if (L.gw) A.tape_gw_in = (const float*)(sb + L.gw);
  int grid = (int)std::max<int64_t>(1, std::min<int64_t>((a->n_paths + 255) / 256, (int64_t)c->n_cu * 16));
  if (a->flags & LT_ATTACHED) {
    A.emit_d = (float*)(sb + L.emit);
    A.hgrad_lds = hgrad_in_lds(c, g->heights, BwdKernel::naive_att, 256, 0, false);
    A.agrad_lds = agrad_in_lds(c, BwdKernel::naive_att, 256, hgrad_lds_bytes(c, A.hgrad_lds));
    if ((st = c->hip(launch_naive_att_bwd(A, grid, c->stream), "naive attached backward")) != LT_OK) return st;
  } else {
    A.agrad_lds = agrad_in_lds(c, BwdKernel::naive, 256, 0);
    A.legrad_lds = legrad_in_lds(c, BwdKernel::naive, 256, agrad_lds_bytes(c, A.agrad_lds));
    if ((st = c->hip(launch_naive_bwd(A, grid, c->stream), "naive backward")) != LT_OK) return st;
  }
  return c->hip(launch_add_le(c->d_acc, g->emitter_L, c->stream), "emitter gradient");
}

lt_status lt_backward_reslrb(lt_ctx* c, const lt_trace_args* a, const lt_params* p, const float* d_image,
                             const void* records, size_t bytes, lt_grads* g) {
  if (!c) return LT_ERR_ARG;
  if (a && !(a->flags & LT_RECORD_RESERVOIR)) return c->fail(LT_ERR_ARG, "ResLRB backward needs LT_RECORD_RESERVOIR args%s");
  if (a && (!records || bytes < side_layout(c, a).total)) return c->fail(LT_ERR_ARG, "reservoir buffer too small%s");
  PassArgs A;
  lt_status st = backward_common(c, a, p, d_image, g, A, a ? side_layout(c, a).total : 0);
  if (st != LT_OK) return st;
  SideLayout L = side_layout(c, a);
  if (a->flags & LT_ATTACHED) {
    A.res_att_in = (const ResRecAtt*)((const char*)records + L.res);
    const int blk = att_replay_block(c, g->heights, c->dsc.stack_n, BwdKernel::reslrb_att, 512);
    int grid = persistent_grid(c, a->n_paths, blk);
    A.hgrad_lds = hgrad_in_lds(c, g->heights, BwdKernel::reslrb_att, blk, stack_lds(c, blk), true);
    A.agrad_lds = agrad_in_lds(c, BwdKernel::reslrb_att, blk, stack_lds(c, blk) + hgrad_lds_bytes(c, A.hgrad_lds));
    if ((st = c->hip(launch_reslrb_att(A, grid, blk, c->stream), "reslrb attached backward")) != LT_OK) return st;
    return c->hip(launch_add_le(c->d_acc, g->emitter_L, c->stream), "emitter gradient");
  }
  A.res_in = (const ResRec*)((const char*)records + L.res);
  const Shape sh = replay_shape(c, BwdKernel::reslrb, a->n_paths);
  A.agrad_lds = sh.agrad_lds;
  A.legrad_lds = legrad_in_lds(c, BwdKernel::reslrb, sh.block, stack_lds(c, sh.block) + agrad_lds_bytes(c, sh.agrad_lds));
  if ((st = c->hip(launch_reslrb_bwd(A, sh.grid, sh.block, c->stream), "reslrb backward")) != LT_OK) return st;
  return c->hip(launch_add_le(c->d_acc, g->emitter_L, c->stream), "emitter gradient");
}

lt_status lt_backward_lrb2(lt_ctx* c, const lt_trace_args* a, const lt_params* p, const float* d_image,
                           const void* records, size_t bytes, lt_grads* g) {
  if (!c) return LT_ERR_ARG;
  if (a && (a->flags & LT_ATTACHED)) return c->fail(LT_ERR_UNSUPPORTED, "the buffered two-pass backward is detached%s");
  if (a && !(a->flags & LT_RECORD_SPLATS)) return c->fail(LT_ERR_ARG, "two-pass backward needs LT_RECORD_SPLATS args%s");
  if (a && (!records || bytes < side_layout(c, a).total)) return c->fail(LT_ERR_ARG, "splat record buffer too small%s");
  PassArgs A;
  lt_status st = backward_common(c, a, p, d_image, g, A, a ? side_layout(c, a).total : 0);
  if (st != LT_OK) return st;
  SideLayout L = side_layout(c, a);
  A.contrib = a->path_contrib;
  A.spl_hdr_in = (const SplatHdr*)((const char*)records + L.spl_hdr);
  A.spl_in = (const SplatRec*)((const char*)records + L.spl);
  const Shape sh = replay_shape(c, BwdKernel::lrb2, a->n_paths);
  A.agrad_lds = sh.agrad_lds;
  A.legrad_lds = legrad_in_lds(c, BwdKernel::lrb2, sh.block, stack_lds(c, sh.block) + agrad_lds_bytes(c, sh.agrad_lds));
  if ((st = c->hip(launch_lrb2_bwd(A, sh.grid, sh.block, c->stream), "two-pass backward")) != LT_OK) return st;
  return c->hip(launch_add_le(c->d_acc, g->emitter_L, c->stream), "emitter gradient");
}

// The LRB-3 backward on the working memory w (see Work).
static lt_status lrb3_enqueue(lt_ctx* c, const lt_trace_args* a, const lt_params* p, const float* d_image,
                              lt_grads* g, const Work& w) {
  PassArgs A;
  lt_status st = backward_common(c, a, p, d_image, g, A, w.hand ? 0 : hand_bytes(c, a), w);
  if (st != LT_OK) return st;
  A.contrib = a->path_contrib;
  const bool att = (a->flags & LT_ATTACHED) != 0;
  if (lrb3_split(c, a)) {
    // pass 2 appends a hand-off entry per connected path; pass 3 replays those
    char* hand = w.hand;
    if (!hand) {
      if ((st = grow(c, &c->d_hand, c->hand_n, hand_bytes(c, a), "the LRB-3 hand-off")) != LT_OK) return st;
      hand = c->d_hand;
    }
    A.hand = reinterpret_cast<Lrb3Hand*>(hand);
    A.hand_att = reinterpret_cast<Lrb3HandAtt*>(hand);
    A.hand_region = hand_region(a->n_paths);
    A.counter3 = w.counter + kCtrBlock;
    A.hand_app = w.counter + 2 * kCtrBlock;
    if ((st = c->hip(launch_fill_u32(A.counter3, 2 * kCtrBlock, 0u, c->stream), "hand-off counter clear")) != LT_OK)
      return st;
    if (att) {
      const int blk2 = 256;
      if ((st = c->hip(launch_lrb3_att_p2(A, persistent_grid(c, a->n_paths, blk2), blk2, c->stream),
                       "lrb3 attached pass 2")) != LT_OK)
        return st;
      // rough conductors: the pass-3 kernel at two waves per SIMD, workgroups of at most 512 threads
      const BwdKernel k3 = A.cond ? BwdKernel::lrb3_att_p3_cond : BwdKernel::lrb3_att_p3;
      const int blk = att_replay_block(c, g->heights, c->dsc.stack_n, k3, A.cond ? 512 : 768);
      A.hgrad_lds = hgrad_in_lds(c, g->heights, k3, blk, stack_lds(c, blk), true);
      A.agrad_lds = agrad_in_lds(c, k3, blk, stack_lds(c, blk) + hgrad_lds_bytes(c, A.hgrad_lds));
      if ((st = c->hip(launch_lrb3_att_p3(A, persistent_grid(c, a->n_paths, blk), blk, c->stream),
                       "lrb3 attached pass 3")) != LT_OK)
        return st;
    } else {
      const int blk = c->tune.block;
      A.agrad_lds = 0;  // pass 2 scatters no albedo gradients
      A.legrad_lds = legrad_in_lds(c, BwdKernel::lrb3_p2, blk, stack_lds(c, blk));
      if ((st = c->hip(launch_lrb3_p2(A, persistent_grid(c, a->n_paths, blk), blk, c->stream), "lrb3 pass 2")) !=
          LT_OK)
        return st;
      const Shape sh = replay_shape(c, BwdKernel::lrb3_p3, a->n_paths);
      A.agrad_lds = sh.agrad_lds;
      A.legrad_lds = 0;  // pass 3 adds no emitter gradients
      if ((st = c->hip(launch_lrb3_p3(A, sh.grid, sh.block, c->stream), "lrb3 pass 3")) != LT_OK) return st;
    }
  } else if (att) {
    // rough conductors: two waves per SIMD, workgroups of at most 512 threads
    const BwdKernel k = A.cond ? BwdKernel::lrb3_att_cond : BwdKernel::lrb3_att;
    const int blk = att_replay_block(c, g->heights, c->dsc.stack_n, k, A.cond ? 512 : 768);
    int grid = persistent_grid(c, a->n_paths, blk);
    A.hgrad_lds = hgrad_in_lds(c, g->heights, k, blk, stack_lds(c, blk), true);
    A.agrad_lds = agrad_in_lds(c, k, blk, stack_lds(c, blk) + hgrad_lds_bytes(c, A.hgrad_lds));
    if ((st = c->hip(launch_lrb3_att(A, grid, blk, c->stream), "lrb3 attached backward")) != LT_OK) return st;
  } else {
    const Shape sh = replay_shape(c, BwdKernel::lrb3, a->n_paths);
    A.agrad_lds = sh.agrad_lds;
    A.legrad_lds = legrad_in_lds(c, BwdKernel::lrb3, sh.block, stack_lds(c, sh.block) + agrad_lds_bytes(c, sh.agrad_lds));
    if ((st = c->hip(launch_lrb3_bwd(A, sh.grid, sh.block, c->stream), "lrb3 backward")) != LT_OK) return st;
  }
  return c->hip(launch_add_le(w.acc, g->emitter_L, c->stream), "emitter gradient");
}

lt_status lt_backward_lrb3(lt_ctx* c, const lt_trace_args* a, const lt_params* p, const float* d_image,
                           lt_grads* g) {
  if (!c) return LT_ERR_ARG;
  return lrb3_enqueue(c, a, p, d_image, g, ctx_work(c));
}

lt_status lt_backward_lrb3_noalloc(lt_ctx* c, const lt_trace_args* a, const lt_params* p, const float* d_image,
                                   lt_grads* g) {
  if (!c) return LT_ERR_ARG;
  if (!c->d_scratch) return c->fail(LT_ERR_UNSUPPORTED, "the static scratch has no address on this device%s");
  if (!a || !p) return c->fail(LT_ERR_ARG, "null args or params%s");
  if (p->guide_w) return c->fail(LT_ERR_UNSUPPORTED, "the no-allocation backward takes no guide (its records are allocated)%s");
  const size_t cap = kScratchBytes - kScratchHand;
  if (a->n_paths >= 1 && hand_bytes(c, a) > cap) {
    char buf[256];
    const size_t entry = (a->flags & LT_ATTACHED) ? sizeof(Lrb3HandAtt) : sizeof(Lrb3Hand);
    std::snprintf(buf, sizeof(buf), "n_paths %lld exceeds the static scratch: at most %zu paths in this form",
                  (long long)a->n_paths, cap / entry);
    c->err = buf;
    return LT_ERR_ARG;
  }
  Work w{reinterpret_cast<unsigned int*>(c->d_scratch + kScratchCounters),
         reinterpret_cast<double*>(c->d_scratch + kScratchAcc), c->d_scratch + kScratchHand, cap};
  return lrb3_enqueue(c, a, p, d_image, g, w);
}

// Camera side: the light-tracing argument checks on the same args with no
// flags, then the camera's own conditions.
static lt_status camera_check(lt_ctx* c, const lt_trace_args* a, const lt_params* p, lt_trace_args& b,
                              lt_params& q) {
  if (!c) return LT_ERR_ARG;
  if (!a || !p) return c->fail(LT_ERR_ARG, "null args or params%s");
  b = *a;
  b.flags = 0;
  b.path_info = nullptr;
  b.path_contrib = nullptr;
  q = *p;
  q.guide_w = nullptr;
  lt_status st = check_args(c, &b, &q);
  if (st != LT_OK) return st;
  if (a->flags & ~(uint32_t)LT_CAMERA_ALL)
    return c->fail(LT_ERR_UNSUPPORTED, "camera samples take LT_CAMERA_ALL only (detached)%s");
  if (c->dsc.em_type == LT_EMIT_DIRECTIONAL)
    return c->fail(LT_ERR_UNSUPPORTED, "camera samples cannot reach a directional emitter%s");
  const int64_t npx = (int64_t)c->dsc.W * c->dsc.H;
  if (a->n_paths % npx != 0) return c->fail(LT_ERR_ARG, "camera samples: n_paths must be a multiple of width*height%s");
  return LT_OK;
}

static void camera_fields(const lt_ctx* c, const lt_trace_args* a, PassArgs& A) {
  A.flags = (a->flags & LT_CAMERA_ALL) ? 1u : 0u;
  A.spp_inv = (float)((double)c->dsc.W * c->dsc.H / (double)a->n_paths);
  A.guide_rec = nullptr;
  A.gtab = nullptr;
}

lt_status lt_camera_trace(lt_ctx* c, const lt_trace_args* a, const lt_params* p, float* image) {
  lt_trace_args b;
  lt_params q;
  lt_status st = camera_check(c, a, p, b, q);
  if (st != LT_OK) return st;
  if (!image) return c->fail(LT_ERR_ARG, "null image%s");
  if ((st = prepare_geometry(c, &q)) != LT_OK) return st;
  PassArgs A = base_args(c, &b, &q);
  camera_fields(c, a, A);
  A.image = image;
  if ((st = c->hip(launch_fill_u32(c->d_counter, kCtrBlock, 0u, c->stream), "counter clear")) != LT_OK) return st;
  if ((st = c->hip(launch_fill_u32(c->d_counter + kCtrStats, 4, 0u, c->stream), "stats clear")) != LT_OK) return st;
  const int blk = c->tune.block;
  return c->hip(launch_camera(A, persistent_grid(c, a->n_paths, blk), blk, c->stream), "camera launch");
}

lt_status lt_camera_backward_prb(lt_ctx* c, const lt_trace_args* a, const lt_params* p, const float* d_image,
                                 lt_grads* g) {
  lt_trace_args b;
  lt_params q;
  lt_status st = camera_check(c, a, p, b, q);
  if (st != LT_OK) return st;
  PassArgs A;
  if ((st = backward_common(c, &b, &q, d_image, g, A, 0)) != LT_OK) return st;
  camera_fields(c, a, A);
  const Shape sh = replay_shape(c, BwdKernel::camera_prb, a->n_paths);
  A.agrad_lds = sh.agrad_lds;
  if ((st = c->hip(launch_camera_prb(A, sh.grid, sh.block, c->stream), "camera backward")) != LT_OK) return st;
  return c->hip(launch_add_le(c->d_acc, g->emitter_L, c->stream), "emitter gradient");
}

lt_status lt_guide_eval(lt_ctx* c, const float* guide_w, const float* x, const float* n, int64_t count,
                        float* out) {
  if (!c) return LT_ERR_ARG;
  if (!guide_w || !x || !n || !out || count < 1 || count >= ((int64_t)1 << 31))
    return c->fail(LT_ERR_ARG, "bad guide eval arguments%s");
  if (!c->has_scene) return c->fail(LT_ERR_STATE, "no scene uploaded%s");
  if (!c->guide_ok) return c->fail(LT_ERR_UNSUPPORTED, "guide kernels could not get their LDS%s");
  lt_status st = guide_pack(c, guide_w);
  if (st != LT_OK) return st;
  GuideArgs G = guide_args(c, guide_w, count);
  G.x = x; G.n = n; G.out = out;
  return c->hip(launch_guide_eval(G, guide_grid(c, count), c->stream), "guide eval");
}

lt_status lt_guide_emit(lt_ctx* c, const lt_trace_args* a, const lt_params* p, const float* path_contrib,
                        lt_guide_sample* out) {
  if (!c) return LT_ERR_ARG;
  if (!a || !p || !out || !p->guide_w) return c->fail(LT_ERR_ARG, "bad guide emit arguments%s");
  if (!c->has_scene) return c->fail(LT_ERR_STATE, "no scene uploaded%s");
  if (a->n_paths < 1 || a->n_paths >= (int64_t)1 << 31) return c->fail(LT_ERR_ARG, "n_paths out of range [1, 2^31)%s");
  if (c->dsc.em_type != LT_EMIT_QUAD) return c->fail(LT_ERR_UNSUPPORTED, "the emission guide needs an area emitter%s");
  if (!c->guide_ok) return c->fail(LT_ERR_UNSUPPORTED, "guide kernels could not get their LDS%s");
  lt_status st = guide_pack(c, p->guide_w);
  if (st != LT_OK) return st;
  GuideArgs G = guide_args(c, p->guide_w, a->n_paths);
  G.seed = a->seed;
  G.samples = reinterpret_cast<float*>(out);
  G.contrib = path_contrib;
  return c->hip(launch_guide_emit(G, guide_grid(c, a->n_paths), c->stream), "guide emit");
}

lt_status lt_guide_vertex_samples(lt_ctx* c, const lt_trace_args* a, const lt_params* p, lt_guide_sample* out) {
  lt_status st = check_args(c, a, p);
  if (st != LT_OK) return st;
  if (!out || !p->guide_w) return c->fail(LT_ERR_ARG, "bad diffuse guide sample arguments%s");
  if (a->flags & (LT_ATTACHED | LT_RECORD_TAPE | LT_RECORD_RESERVOIR | LT_RECORD_SPLATS | LT_SPLAT_SELECTED))
    return c->fail(LT_ERR_ARG, "diffuse guide samples take a plain detached pass (flags LT_GUIDE_DIFFUSE only)%s");
  lt_trace_args e = *a;
  e.flags = LT_GUIDE_DIFFUSE;
  if ((st = check_cap(c, guide_bytes(&e, p))) != LT_OK) return st;
  if ((st = prepare_geometry(c, p)) != LT_OK) return st;
  PassArgs A = base_args(c, &e, p);
  A.gsamp = reinterpret_cast<float*>(out);
  if ((st = guide_prepass(c, &e, p, A)) != LT_OK) return st;
  if ((st = c->hip(launch_fill_u32(c->d_counter, kCtrBlock, 0u, c->stream), "counter clear")) != LT_OK) return st;
  int grid = persistent_grid(c, a->n_paths, c->tune.block);
  return c->hip(launch_trace_gsamples(A, grid, c->tune.block, c->stream), "diffuse guide samples");
}

lt_status lt_guide_grad(lt_ctx* c, const float* guide_w, const lt_guide_sample* samples, int64_t count,
                        float* grad, float* loss) {
  if (!c) return LT_ERR_ARG;
  if (!guide_w || !samples || !grad || count < 1 || count >= ((int64_t)1 << 31))
    return c->fail(LT_ERR_ARG, "bad guide gradient arguments%s");
  if (!c->has_scene) return c->fail(LT_ERR_STATE, "no scene uploaded%s");
  if (!c->guide_ok) return c->fail(LT_ERR_UNSUPPORTED, "guide kernels could not get their LDS%s");
  int grid = (int)std::min<int64_t>((count + 63) / 64, 1024);
  lt_status st = check_cap(c, (size_t)grid * guide_partial_floats() * sizeof(float));
  if (st != LT_OK) return st;
  if ((st = grow(c, &c->d_gpart, c->gpart_n, (size_t)1024 * guide_partial_floats(), "guide partial sums")) != LT_OK)
    return st;
  if ((st = guide_pack(c, guide_w)) != LT_OK) return st;
  GuideArgs G = guide_args(c, guide_w, count);
  G.samples = const_cast<float*>(reinterpret_cast<const float*>(samples));
  G.partial = c->d_gpart;
  if ((st = c->hip(launch_guide_grad(G, grid, c->stream), "guide gradient")) != LT_OK) return st;
  return c->hip(launch_guide_reduce(c->d_gpart, grid, grad, loss, c->stream), "guide reduce");
}

lt_status lt_guide_adam(lt_ctx* c, float* w, const float* grad, float* m, float* v, int32_t step, float lr,
                        float beta1, float beta2, float eps) {
  if (!c) return LT_ERR_ARG;
  if (!w || !grad || !m || !v || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
    return c->fail(LT_ERR_ARG, "bad Adam arguments%s");
  float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
  float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
  return c->hip(launch_guide_adam(w, grad, m, v, LT_GUIDE_NPARAMS, lr, beta1, beta2, eps, c1, c2, c->stream),
                "guide adam");
}

lt_status lt_guide_train_step(lt_ctx* c, const lt_trace_args* a, float* guide_w, const float* path_contrib,
                              lt_guide_sample* samples, int64_t n_samples, float* grad, float* m, float* v,
                              float* loss, int32_t step, float lr, float beta1, float beta2, float eps) {
  if (!c) return LT_ERR_ARG;
  // everything the three steps check, before any of them enqueues
  if (!a || !guide_w || !samples || !grad || !m || !v || n_samples < 1 || step < 1 || !(lr > 0.f) ||
      !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
    return c->fail(LT_ERR_ARG, "bad guide training-step arguments%s");
  if (!c->has_scene) return c->fail(LT_ERR_STATE, "no scene uploaded%s");
  if (a->n_paths < 1 || a->n_paths >= (int64_t)1 << 31) return c->fail(LT_ERR_ARG, "n_paths out of range [1, 2^31)%s");
  if (c->dsc.em_type != LT_EMIT_QUAD) return c->fail(LT_ERR_UNSUPPORTED, "the emission guide needs an area emitter%s");
  if (!c->guide_ok) return c->fail(LT_ERR_UNSUPPORTED, "guide kernels could not get their LDS%s");
  lt_trace_args e = *a;
  e.n_paths = std::min<int64_t>(a->n_paths, n_samples);
  int grid = (int)std::min<int64_t>((e.n_paths + 63) / 64, 1024);
  lt_status st = check_cap(c, (size_t)grid * guide_partial_floats() * sizeof(float));
  if (st != LT_OK) return st;
  lt_params p{};
  p.guide_w = guide_w;
  if ((st = lt_guide_emit(c, &e, &p, path_contrib, samples)) != LT_OK) return st;
  if ((st = lt_guide_grad(c, guide_w, samples, e.n_paths, grad, loss)) != LT_OK) return st;
  return lt_guide_adam(c, guide_w, grad, m, v, step, lr, beta1, beta2, eps);
}

}  // extern "C"

// ============================================================== batches
#include <map>
#include <fstream>
#include <sstream>

struct lt_batch {
  int device = 0;
  hipStream_t stream = nullptr;       // caller's stream: eager steps and graph launches
  hipStream_t cap = nullptr;          // the runner's own stream, for capture (the null stream cannot be)
  std::string err;
  lt_tuning tune{256, 4, 1, 0};
  int n_cu = 256;
  std::string arch;
  // device tables: trace [n], detached backward [n_det], attached backward [n_att]
  PassArgs* d_tab = nullptr;
  size_t tab_cap = 0;                 // PassArgs entries allocated
  unsigned int* d_cnt = nullptr;      // work counters, a block per pass of each instance [2n][kCtrBlock]
  double* d_acc = nullptr;            // per instance: emitter gradient (3) + loss (1)
  size_t inst_cap = 0;
  char* d_hand = nullptr;             // LRB-3 hand-off of the solo attached instances, one at a time
  size_t hand_cap = 0;                // bytes
  unsigned int* d_hcnt = nullptr;     // LRB-3 pass-3 and append counters of the solo instances [n][2][kCtrBlock]
  // captured step
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<char> key;              // the instance set the graph was captured for

  lt_status fail(lt_status s, const char* msg) { err = msg; return s; }
  lt_status hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return LT_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return LT_ERR_HIP;
  }
  void drop_graph() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    exec = nullptr; graph = nullptr; key.clear();
  }
};

namespace {

// Instances of at least this many paths run their backward as launches of
// their own: attached ones the two-kernel LRB-3 of the single-instance call
// (three waves per SIMD against the multi-entry kernel's two), detached ones
// the single-instance kernel's body (the multi-entry kernel spills more;
// 48-instance step, 20 detached of 1M-32M paths: 183.5 -> 149.6 ms).  At that
// size a launch's tail and gap are small against its work.
constexpr int64_t kSoloPaths = (int64_t)1 << 20;
// Instances of at least this many paths run their forward as a launch of its
// own, the single-instance kernel at five waves per SIMD; smaller ones gain
// more from sharing one launch's tail.
constexpr int64_t kSoloTracePaths = (int64_t)1 << 22;

struct BatchPlan {
  // [n trace: n_bt batched, then the solo ones][n_det detached][n_att attached][n_solo attached]
  // [n_solo_det detached], the solo ones a launch each
  std::vector<PassArgs> tab;
  std::vector<int> trace_pos;       // table position of each instance's forward entry
  std::vector<int> solo_trace;      // instances whose forward runs on its own
  std::vector<int> solo_trace_shape;  // per solo forward launch: block, grid, heightfield
  int n_bt = 0;                     // batched forward entries (the table's first)
  std::vector<int> det, att, solo, solo_det;  // instance indices of each backward kind
  int n = 0, stack_n = 1;      // traversal stack entries per lane, the same for every entry
  bool det_hf = false;         // some batched detached entry has a heightfield
  size_t det_lds = 0, att_lds = 0;  // LDS bytes past the stacks for gradient copies, per launch
  std::vector<size_t> solo_lds;     // the same for each solo launch
  std::vector<int> solo_block;      // workgroup size of each solo launch
  std::vector<int> solo_det_shape;  // per solo detached launch: block, grid, LDS bytes past the stacks, heightfield
};

// Largest of the sizes the instances ask for that fits next to the traversal
// stacks and costs the batched kernel no resident workgroups per CU (0 if
// none does).  Residency only falls as the size grows, so the first fit from
// the top is the answer.
size_t batch_lds_budget(BwdKernel k, int block, size_t stack, size_t lds_max, std::vector<size_t> sizes) {
  std::sort(sizes.begin(), sizes.end());
  sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
  const int base = resident_groups(k, block, stack);
  for (auto it = sizes.rbegin(); it != sizes.rend() && *it > 0; ++it) {
    if (stack + *it > lds_max) continue;
    int r = resident_groups(k, block, stack + *it);
    if (r > 0 && r >= base) return *it;
  }
  return 0;
}

lt_status batch_check(lt_batch* b, const lt_instance* inst, int n) {
  if (!inst || n < 1 || n > 4096) return b->fail(LT_ERR_ARG, "need 1..4096 instances");
  for (int i = 0; i < n; ++i) {
    const lt_instance& I = inst[i];
    lt_ctx* c = I.ctx;
    if (!c) return b->fail(LT_ERR_ARG, "instance without a context");
    if (c->device != b->device) return b->fail(LT_ERR_ARG, "instance context on another device");
    if (I.args.flags & ~(uint32_t)LT_ATTACHED) return b->fail(LT_ERR_UNSUPPORTED, "batches take flags 0 or LT_ATTACHED only");
    if ((I.args.flags & LT_ATTACHED) && c->has_conductor)
      return b->fail(LT_ERR_UNSUPPORTED, "attached batches take no rough-conductor scenes");
    if (I.args.path_sig || I.args.path_info || I.args.path_contrib)
      return b->fail(LT_ERR_UNSUPPORTED, "batches take no signatures, info or contributions");
    lt_status st = check_args(c, &I.args, &I.params);
    if (st != LT_OK) { b->err = "instance " + std::to_string(i) + ": " + c->err; return st; }
    if (!I.target || !I.image || !I.d_image || !I.loss || !I.grads.albedo)
      return b->fail(LT_ERR_ARG, "instance buffers (target, image, d_image, loss, grads.albedo) are required");
  }
  return LT_OK;
}

// Allocations every step needs, made before any capture.
lt_status batch_reserve(lt_batch* b, const lt_instance* inst, int n) {
  size_t need = (size_t)2 * n;
  if (b->tab_cap < need) {
    hipFree(b->d_tab); b->d_tab = nullptr; b->tab_cap = 0;
    if (hipMalloc((void**)&b->d_tab, need * sizeof(PassArgs)) != hipSuccess) {
      (void)hipGetLastError();
      return b->fail(LT_ERR_OOM, "out of device memory for the instance table");
    }
    b->tab_cap = need;
  }
  if (b->inst_cap < (size_t)n) {
    hipFree(b->d_cnt); hipFree(b->d_acc); hipFree(b->d_hcnt);
    b->d_cnt = nullptr; b->d_acc = nullptr; b->d_hcnt = nullptr; b->inst_cap = 0;
    if (hipMalloc((void**)&b->d_cnt, (size_t)2 * n * kCtrBlock * sizeof(unsigned int)) != hipSuccess ||
        hipMalloc((void**)&b->d_acc, (size_t)4 * n * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&b->d_hcnt, (size_t)n * 2 * kCtrBlock * sizeof(unsigned int)) != hipSuccess) {
      (void)hipGetLastError();
      return b->fail(LT_ERR_OOM, "out of device memory for the batch counters");
    }
    b->inst_cap = n;
  }
  size_t hand = 0;  // the largest solo instance's hand-off
  for (int i = 0; i < n; ++i)
    if ((inst[i].args.flags & LT_ATTACHED) && inst[i].args.n_paths >= kSoloPaths)
      hand = std::max(hand, (size_t)kWorkClasses * hand_region(inst[i].args.n_paths) * sizeof(Lrb3HandAtt));
  if (b->hand_cap < hand) {
    hipFree(b->d_hand); b->d_hand = nullptr; b->hand_cap = 0;
    if (hipMalloc((void**)&b->d_hand, hand) != hipSuccess) {
      (void)hipGetLastError();
      return b->fail(LT_ERR_OOM, "out of device memory for the LRB-3 hand-off");
    }
    b->hand_cap = hand;
  }
  for (int i = 0; i < n; ++i) {
    lt_ctx* c = inst[i].ctx;
    if (!inst[i].params.guide_w) continue;
    lt_status st = grow(c, &c->d_grec, c->grec_n, (size_t)inst[i].args.n_paths, "guided emission records");
    if (st == LT_OK && !c->d_gpack && hipMalloc(&c->d_gpack, guide_packed_bytes()) != hipSuccess) {
      (void)hipGetLastError();
      c->d_gpack = nullptr;
      st = LT_ERR_OOM;
    }
    if (st != LT_OK) return b->fail(st, "out of device memory for the guide");
  }
  return LT_OK;
}

BatchPlan batch_plan(lt_batch* b, const lt_instance* inst, int n, int64_t path_div) {
  BatchPlan P;
  P.n = n;
  P.tab.resize((size_t)2 * n);
  for (int i = 0; i < n; ++i) {
    const lt_instance& I = inst[i];
    lt_ctx* c = I.ctx;
    lt_trace_args a = I.args;
    if (path_div > 1) a.n_paths = std::max<int64_t>(std::min<int64_t>(a.n_paths, 65536), a.n_paths / path_div);
    PassArgs A = base_args(c, &a, &I.params);
    A.hgrad_lds = 0;
    A.guide_rec = I.params.guide_w ? c->d_grec : nullptr;
    A.stats = nullptr;
    P.stack_n = std::max(P.stack_n, c->dsc.stack_n);
    PassArgs T = A;
    T.image = I.image;
    T.counter = b->d_cnt + (size_t)i * kCtrBlock;
    P.tab[i] = T;
    PassArgs B = A;
    B.dI = I.d_image;
    B.g_albedo = I.grads.albedo;
    B.g_heights = I.grads.heights;
    B.g_nmap = (I.args.flags & LT_ATTACHED) ? I.grads.normal_map : nullptr;
    B.g_Le_acc = b->d_acc + 4 * i;
    B.g_le_tex = c->dsc.em_tex_res > 0 ? I.grads.emitter_L : nullptr;
    B.counter = b->d_cnt + (size_t)(n + i) * kCtrBlock;
    // by the caller's path count, so the autotuner's shortened steps keep the plan's shape
    const bool big = I.args.n_paths >= kSoloPaths;
    ((a.flags & LT_ATTACHED) ? (big ? P.solo : P.att) : (big ? P.solo_det : P.det)).push_back(i);
    P.tab[n + i] = B;  // reordered below
  }
  // Gradient copies in LDS.  Every entry lays its LDS out past stacks of the
  // batch's common depth, so no instance's copies overlap the stacks of waves
  // still on another instance; the copies of one instance are flushed
  // (workgroup barrier) before its waves move on.
  auto tex_bytes = [&](const lt_ctx* c) -> size_t {
    size_t t = (size_t)c->dsc.n_tex * c->dsc.tex_res * c->dsc.tex_res * 3 * sizeof(float);
    return b->tune.lds_grad && t <= 48 * 1024 ? t : 0;
  };
  auto hf_bytes = [&](const lt_instance& I) -> size_t {
    int G = I.ctx->dsc.hf_G;
    return I.grads.heights && G >= 2 ? (size_t)G * G * sizeof(float) : 0;
  };
  std::vector<size_t> dsz, asz;
  for (int i : P.det) dsz.push_back(tex_bytes(inst[i].ctx));
  for (int i : P.att) {
    size_t t = tex_bytes(inst[i].ctx);
    size_t h = hf_bytes(inst[i]);
    asz.push_back(h); asz.push_back(t);
    if (h && t) asz.push_back(h + t);
  }
  const size_t lds_max = (size_t)inst[0].ctx->lds_max;
  if (!P.det.empty())
    P.det_lds = batch_lds_budget(BwdKernel::lrb3_batch, b->tune.block, (size_t)P.stack_n * b->tune.block * sizeof(int),
                                 lds_max, dsz);
  if (!P.att.empty())
    P.att_lds = batch_lds_budget(BwdKernel::lrb3_att_batch, 256, (size_t)P.stack_n * 256 * sizeof(int), lds_max, asz);
  for (auto& e : P.tab) e.sc.stack_n = P.stack_n;
  for (int i : P.det) {
    size_t t = tex_bytes(inst[i].ctx);
    P.tab[n + i].agrad_lds = t && t <= P.det_lds;
    P.det_hf = P.det_hf || inst[i].ctx->dsc.hf_G >= 2;
  }
  // a solo detached instance takes the single-instance call's launch shape
  // (its LDS copy only where the batch's tuning allows copies)
  for (int i : P.solo_det) {
    PassArgs& B = P.tab[n + i];
    const lt_ctx* c = inst[i].ctx;
    const Shape sh = b->tune.lds_grad ? replay_shape(c, BwdKernel::lrb3_entry, B.n_paths, P.stack_n)
                                      : Shape{c->tune.block, persistent_grid(c, B.n_paths, c->tune.block), 0};
    B.agrad_lds = sh.agrad_lds;
    P.solo_det_shape.insert(P.solo_det_shape.end(),
                            {sh.block, sh.grid, sh.agrad_lds ? (int)(B.n_texels * 3 * sizeof(float)) : 0,
                             c->dsc.hf_G >= 2 ? 1 : 0});
  }
  for (int i : P.att) {
    PassArgs& B = P.tab[n + i];
    size_t h = hf_bytes(inst[i]), t = tex_bytes(inst[i].ctx);
    B.hgrad_lds = h && h <= P.att_lds;
    B.agrad_lds = t && t + (B.hgrad_lds ? h : 0) <= P.att_lds;
  }
  // a solo instance runs the single-instance call's two kernels: pass 3 takes
  // that call's workgroup size and each copy that fits and costs it no
  // resident workgroups; the hand-off goes through the batch's buffer
  for (size_t k = 0; k < P.solo.size(); ++k) {
    const int i = P.solo[k];
    PassArgs& B = P.tab[n + i];
    B.hand_att = reinterpret_cast<Lrb3HandAtt*>(b->d_hand);
    B.counter3 = b->d_hcnt + k * 2 * kCtrBlock;
    B.hand_app = B.counter3 + kCtrBlock;
    B.hand_region = hand_region(B.n_paths);
    const int blk = att_replay_block(inst[i].ctx, inst[i].grads.heights, P.stack_n, BwdKernel::lrb3_att_p3_entry, 768);
    const size_t stack = (size_t)P.stack_n * blk * sizeof(int);
    auto free_of_cost = [&](size_t extra) {
      if (stack + extra > lds_max) return false;
      int r = resident_groups(BwdKernel::lrb3_att_p3_entry, blk, stack + extra);
      return r > 0 && r >= resident_groups(BwdKernel::lrb3_att_p3_entry, blk, stack);
    };
    size_t h = hf_bytes(inst[i]), t = tex_bytes(inst[i].ctx);
    B.hgrad_lds = h && free_of_cost(h);
    size_t hb = B.hgrad_lds ? h : 0;
    B.agrad_lds = t && free_of_cost(hb + t);
    P.solo_lds.push_back(hb + (B.agrad_lds ? t : 0));
    P.solo_block.push_back(blk);
  }
  // forward entries: the batched ones first, then the solo ones
  std::vector<PassArgs> fw;
  P.trace_pos.assign(n, 0);
  for (int i = 0; i < n; ++i)
    if (inst[i].args.n_paths < kSoloTracePaths) { P.trace_pos[i] = (int)fw.size(); fw.push_back(P.tab[i]); }
  P.n_bt = (int)fw.size();
  for (int i = 0; i < n; ++i)
    if (inst[i].args.n_paths >= kSoloTracePaths) {
      const lt_ctx* c = inst[i].ctx;
      P.trace_pos[i] = (int)fw.size();
      fw.push_back(P.tab[i]);
      P.solo_trace.push_back(i);
      P.solo_trace_shape.insert(P.solo_trace_shape.end(), {c->tune.block, persistent_grid(c, P.tab[i].n_paths,
                                                           c->tune.block), c->dsc.hf_G >= 2 ? 1 : 0});
    }
  for (int k = 0; k < n; ++k) P.tab[k] = fw[k];
  // backward entries: detached ones first, then attached ones, then solo ones
  std::vector<PassArgs> bw;
  for (int i : P.det) bw.push_back(P.tab[n + i]);
  for (int i : P.att) bw.push_back(P.tab[n + i]);
  for (int i : P.solo) bw.push_back(P.tab[n + i]);
  for (int i : P.solo_det) bw.push_back(P.tab[n + i]);
  for (int k = 0; k < n; ++k) P.tab[n + k] = bw[k];
  return P;
}

// Everything one step launches, in order on stream s (capturable: fills, no
// memsets, no allocation).  The instance contexts enqueue on s meanwhile and
// are left on the caller's stream.
lt_status batch_enqueue_on(lt_batch* b, const lt_instance* inst, const BatchPlan& P, hipStream_t s) {
  const int n = P.n;
  for (int i = 0; i < n; ++i) {
    const lt_instance& I = inst[i];
    lt_ctx* c = I.ctx;
    c->stream = s;
    lt_status st = prepare_geometry(c, &I.params);
    if (st != LT_OK) return b->fail(st, c->err.c_str());
    if (I.params.guide_w) {
      if ((st = guide_pack(c, I.params.guide_w)) != LT_OK) return b->fail(st, c->err.c_str());
      const int64_t np = P.tab[P.trace_pos[i]].n_paths;
      GuideArgs G = guide_args(c, I.params.guide_w, np);
      G.seed_ptr = &b->d_tab[P.trace_pos[i]].seed;  // the seed as updated before every replay
      G.rec = c->d_grec;
      if ((st = c->hip(launch_guide_emit(G, guide_grid(c, np), s), "guide emit")) != LT_OK)
        return b->fail(st, c->err.c_str());
    }
    size_t npix = (size_t)c->dsc.W * c->dsc.H * 3;
    if ((st = b->hip(launch_fill_f32(I.image, npix, 0.f, s), "image clear")) != LT_OK) return st;
  }
  lt_status st;
  if ((st = b->hip(launch_fill_u32(b->d_cnt, (size_t)2 * n * kCtrBlock, 0u, s), "counter clear")) != LT_OK) return st;
  if ((st = b->hip(launch_fill_f64(b->d_acc, (size_t)4 * n, 0.0, s), "accumulator clear")) != LT_OK) return st;
  int grid = (int)std::max<int64_t>(1, (int64_t)b->n_cu * b->tune.blocks_per_cu);
  if (P.n_bt && (st = b->hip(launch_trace_batch(b->d_tab, P.n_bt, P.stack_n, grid, b->tune.block, s),
                             "batched trace")) != LT_OK)
    return st;
  for (size_t k = 0; k < P.solo_trace.size(); ++k) {
    const int* sh = P.solo_trace_shape.data() + 3 * k;
    if ((st = b->hip(launch_trace_entry(b->d_tab + P.trace_pos[P.solo_trace[k]], sh[2] != 0, P.stack_n, sh[1],
                                        sh[0], s), "trace")) != LT_OK)
      return st;
  }
  for (int i = 0; i < n; ++i) {
    const lt_instance& I = inst[i];
    size_t npix = (size_t)I.ctx->dsc.W * I.ctx->dsc.H * 3;
    if ((st = b->hip(launch_loss(I.image, I.target, npix, I.d_image, b->d_acc + 4 * i + 3, I.loss, s), "loss")) != LT_OK)
      return st;
  }
  const int nd = (int)P.det.size(), na = (int)P.att.size();
  if (nd && (st = b->hip(launch_lrb3_batch(b->d_tab + n, nd, P.det_hf, P.stack_n, P.det_lds, grid, b->tune.block, s),
                         "batched backward")) != LT_OK)
    return st;
  if (na) {
    int grid_att = (int)std::max<int64_t>(1, (int64_t)b->n_cu * b->tune.blocks_per_cu * b->tune.block / 256);
    if ((st = b->hip(launch_lrb3_att_batch(b->d_tab + n + nd, na, P.stack_n, P.att_lds, grid_att, s),
                     "batched attached backward")) != LT_OK)
      return st;
  }
  if (!P.solo.empty() &&
      (st = b->hip(launch_fill_u32(b->d_hcnt, P.solo.size() * 2 * kCtrBlock, 0u, s), "hand-off counter clear")) != LT_OK)
    return st;
  for (size_t k = 0; k < P.solo.size(); ++k) {
    const int e = n + nd + na + (int)k;
    const lt_ctx* c = inst[P.solo[k]].ctx;
    const int grid2 = persistent_grid(c, P.tab[e].n_paths, 256);
    const int grid3 = persistent_grid(c, P.tab[e].n_paths, P.solo_block[k]);
    if ((st = b->hip(launch_lrb3_att_split_entry(b->d_tab + e, P.stack_n, P.solo_lds[k], grid2, grid3,
                                                 P.solo_block[k], s),
                     "attached backward")) != LT_OK)
      return st;
  }
  for (size_t k = 0; k < P.solo_det.size(); ++k) {
    const int e = n + nd + na + (int)P.solo.size() + (int)k;
    const int* sh = P.solo_det_shape.data() + 4 * k;
    if ((st = b->hip(launch_lrb3_entry(b->d_tab + e, sh[3] != 0, P.stack_n, (size_t)sh[2], sh[1], sh[0], s),
                     "detached backward")) != LT_OK)
      return st;
  }
  for (int i = 0; i < n; ++i)
    if ((st = b->hip(launch_add_le(b->d_acc + 4 * i, inst[i].grads.emitter_L, s), "emitter gradient")) != LT_OK)
      return st;
  return LT_OK;
}

lt_status batch_enqueue(lt_batch* b, const lt_instance* inst, const BatchPlan& P, hipStream_t s) {
  lt_status st = batch_enqueue_on(b, inst, P, s);
  for (int i = 0; i < P.n; ++i) inst[i].ctx->stream = b->stream;
  return st;
}

// Identity of a step for graph reuse: the instances (all but the seeds), the
// tuning, the plan's solo launches and its LDS sizes (a scene uploaded again
// into an instance's context may change them).
std::vector<char> batch_key(const lt_batch* b, const lt_instance* inst, int n, const BatchPlan& P) {
  std::vector<lt_instance> v(inst, inst + n);
  for (auto& I : v) I.args.seed = 0;
  std::vector<char> k((const char*)v.data(), (const char*)(v.data() + n));
  const char* t = (const char*)&b->tune;
  k.insert(k.end(), t, t + sizeof(lt_tuning));
  const size_t sz[6] = {(size_t)P.stack_n, P.det_lds, P.att_lds, P.solo.size(), P.solo_det.size(), (size_t)P.det_hf};
  k.insert(k.end(), (const char*)sz, (const char*)(sz + 6));
  k.insert(k.end(), (const char*)P.solo_det.data(), (const char*)(P.solo_det.data() + P.solo_det.size()));
  k.insert(k.end(), (const char*)P.solo_trace.data(), (const char*)(P.solo_trace.data() + P.solo_trace.size()));
  k.insert(k.end(), (const char*)P.solo_trace_shape.data(),
           (const char*)(P.solo_trace_shape.data() + P.solo_trace_shape.size()));
  k.insert(k.end(), (const char*)P.solo_det_shape.data(),
           (const char*)(P.solo_det_shape.data() + P.solo_det_shape.size()));
  k.insert(k.end(), (const char*)P.solo.data(), (const char*)(P.solo.data() + P.solo.size()));
  k.insert(k.end(), (const char*)P.solo_lds.data(), (const char*)(P.solo_lds.data() + P.solo_lds.size()));
  k.insert(k.end(), (const char*)P.solo_block.data(), (const char*)(P.solo_block.data() + P.solo_block.size()));
  return k;
}

lt_status batch_run(lt_batch* b, const lt_instance* inst, int n, bool use_graph, int64_t path_div) {
  lt_status st = batch_check(b, inst, n);
  if (st != LT_OK) return st;
  if (hipSetDevice(b->device) != hipSuccess) return b->fail(LT_ERR_HIP, "hipSetDevice failed");
  if ((st = batch_reserve(b, inst, n)) != LT_OK) return st;
  BatchPlan P = batch_plan(b, inst, n, path_div);
  // the tables (seeds included) go first in stream order, outside any graph
  if ((st = b->hip(hipMemcpyAsync(b->d_tab, P.tab.data(), P.tab.size() * sizeof(PassArgs), hipMemcpyHostToDevice,
                                  b->stream), "table upload")) != LT_OK)
    return st;
  if (!use_graph) return batch_enqueue(b, inst, P, b->stream);
  std::vector<char> key = batch_key(b, inst, n, P);
  if (!b->exec || key != b->key) {
    b->drop_graph();
    if (!b->cap && (st = b->hip(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "capture stream")) != LT_OK)
      return st;
    if ((st = b->hip(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed), "begin capture")) != LT_OK) return st;
    lt_status est = batch_enqueue(b, inst, P, b->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (est != LT_OK) { if (g) hipGraphDestroy(g); return est; }
    if (e != hipSuccess) return b->hip(e, "end capture");
    b->graph = g;
    if ((st = b->hip(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate")) != LT_OK) {
      b->drop_graph();
      return st;
    }
    b->key = key;
  }
  return b->hip(hipGraphLaunch(b->exec, b->stream), "graph launch");
}

// JSON cache of tuning choices: one entry per line,
//   "key": {"block": B, "blocks_per_cu": K, "ms": T},
std::map<std::string, std::string> cache_read(const char* path) {
  std::map<std::string, std::string> m;
  if (!path) return m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    size_t a = line.find('"'), b = a == std::string::npos ? a : line.find('"', a + 1);
    size_t c = line.find('{'), d = line.rfind('}');
    if (a == std::string::npos || b == std::string::npos || c == std::string::npos || d == std::string::npos || c > d)
      continue;
    m[line.substr(a + 1, b - a - 1)] = line.substr(c, d - c + 1);
  }
  return m;
}
bool cache_field(const std::string& obj, const char* name, double& v) {
  std::string k = std::string("\"") + name + "\"";
  size_t p = obj.find(k);
  if (p == std::string::npos) return false;
  p = obj.find(':', p);
  if (p == std::string::npos) return false;
  v = std::strtod(obj.c_str() + p + 1, nullptr);
  return true;
}
void cache_write(const char* path, const std::map<std::string, std::string>& m) {
  if (!path) return;
  std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    f << "{\n";
    size_t i = 0;
    for (auto& kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++i < m.size() ? ",\n" : "\n");
    f << "}\n";
  }
  std::rename(tmp.c_str(), path);
}

}  // namespace

extern "C" {

lt_status lt_batch_create(int device, void* stream, lt_batch** out) {
  if (!out) return LT_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LT_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return LT_ERR_HIP;
  lt_batch* b = new (std::nothrow) lt_batch();
  if (!b) return LT_ERR_OOM;
  b->device = device;
  b->stream = (hipStream_t)stream;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    if (prop.multiProcessorCount > 0) b->n_cu = prop.multiProcessorCount;
    b->arch = prop.gcnArchName;
  }
  *out = b;
  return LT_OK;
}

void lt_batch_destroy(lt_batch* b) {
  if (!b) return;
  hipSetDevice(b->device);
  b->drop_graph();
  if (b->cap) hipStreamDestroy(b->cap);
  hipFree(b->d_tab);
  hipFree(b->d_cnt);
  hipFree(b->d_acc);
  hipFree(b->d_hcnt);
  hipFree(b->d_hand);
  delete b;
}

const char* lt_batch_last_error(const lt_batch* b) { return b ? b->err.c_str() : "null batch"; }

lt_status lt_batch_set_tuning(lt_batch* b, const lt_tuning* t) {
  if (!b) return LT_ERR_ARG;
  if (!t) { b->tune = lt_tuning{256, 4, 1, 0}; return LT_OK; }
  if (t->block < 64 || t->block > 1024 || (t->block % 64) != 0)
    return b->fail(LT_ERR_ARG, "block must be 64..1024, a multiple of 64");
  if (t->blocks_per_cu < 1 || t->blocks_per_cu > 64) return b->fail(LT_ERR_ARG, "blocks_per_cu must be 1..64");
  b->tune = *t;
  return LT_OK;
}

lt_status lt_batch_get_tuning(const lt_batch* b, lt_tuning* out) {
  if (!b || !out) return LT_ERR_ARG;
  *out = b->tune;
  return LT_OK;
}

lt_status lt_batch_step(lt_batch* b, const lt_instance* inst, int32_t n, int32_t use_graph) {
  if (!b) return LT_ERR_ARG;
  return batch_run(b, inst, n, use_graph != 0, 1);
}

lt_status lt_batch_autotune(lt_batch* b, const lt_instance* inst, int32_t n, const char* cache_path, lt_tuning* out) {
  if (!b) return LT_ERR_ARG;
  lt_status st = batch_check(b, inst, n);
  if (st != LT_OK) return st;
  int64_t total = 0;
  int n_att = 0;
  for (int i = 0; i < n; ++i) {
    total += inst[i].args.n_paths;
    n_att += (inst[i].args.flags & LT_ATTACHED) ? 1 : 0;
  }
  char key[256];
  const int32_t lg = b->tune.lds_grad;  // kept: the trials choose the launch shape only
  std::snprintf(key, sizeof(key), "%s|cu%d|n%d|att%d|paths%lld|lds%d", b->arch.c_str(), b->n_cu, n, n_att,
                (long long)total, (int)lg);
  auto cache = cache_read(cache_path);
  auto it = cache.find(key);
  double bl = 0, bpc = 0;
  if (it != cache.end() && cache_field(it->second, "block", bl) && cache_field(it->second, "blocks_per_cu", bpc)) {
    lt_tuning t{(int32_t)bl, (int32_t)bpc, lg, 0};
    if ((st = lt_batch_set_tuning(b, &t)) == LT_OK && out) *out = t;
    return st;
  }
  static const int blocks[] = {128, 256, 512};
  static const int per_cu[] = {2, 4, 8};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return b->fail(LT_ERR_HIP, "event create");
  lt_tuning best{256, 4, lg, 0};
  float best_ms = 1e30f;
  const lt_tuning saved = b->tune;
  for (int blk : blocks)
    for (int k : per_cu) {
      b->tune = lt_tuning{blk, k, lg, 0};
      float ms = 0.f;
      for (int rep = 0; rep < 3 && st == LT_OK; ++rep) {
        hipEventRecord(e0, b->stream);
        st = batch_run(b, inst, n, false, 16);
        hipEventRecord(e1, b->stream);
        if (st == LT_OK && hipEventSynchronize(e1) != hipSuccess) st = b->fail(LT_ERR_HIP, "trial step");
        float t = 0.f;
        if (st == LT_OK && rep > 0 && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms += t;
      }
      if (st != LT_OK) break;
      if (ms < best_ms) { best_ms = ms; best = b->tune; }
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  b->tune = saved;
  if (st != LT_OK) return st;
  if ((st = lt_batch_set_tuning(b, &best)) != LT_OK) return st;
  char val[160];
  std::snprintf(val, sizeof(val), "{\"block\": %d, \"blocks_per_cu\": %d, \"ms\": %.3f}", best.block,
                best.blocks_per_cu, best_ms / 2.0f);
  cache[key] = val;
  cache_write(cache_path, cache);
  if (out) *out = best;
  return LT_OK;
}

}  // extern "C"
