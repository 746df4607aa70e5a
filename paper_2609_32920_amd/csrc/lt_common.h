// Layouts shared by the host runtime and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace lt {

constexpr int kStackMax = 32;     // BVH traversal stack entries per lane (LDS)
constexpr int kMaxDepth = 64;     // largest max_depth accepted
constexpr float kEps = 1e-4f;     // ray-origin offset along the geometric normal
constexpr float kTmin = 1e-4f;    // closest/any-hit lower bound

// Work counters of a pass: eight, counter c dealing out the path indices
// p = 8k + c, each on a 128-byte line of its own; a context's counter area
// holds three such blocks (the pass's; LRB-3 pass 3's; pass 2's append
// counters of the hand-off, one per class) and, after them, the two 64-bit
// statistics.
constexpr int kWorkClasses = 8;
constexpr int kCtrStride = 32;                        // u32 from one counter to the next
constexpr int kCtrBlock = kWorkClasses * kCtrStride;  // u32 of one pass's counters (1 KB)
constexpr int kCtrStats = 3 * kCtrBlock;              // u32 index of the statistics (byte 3072)
constexpr int kCtrBytes = 4096;                       // bytes of a counter area

// Two-child BVH node, 64 bytes: both child boxes arrive with one fetch.
// count > 0: the child is a leaf holding `count` triangles from `child`;
// count == 0: `child` is an inner node index; child < 0: empty.
struct alignas(16) Node {
  float lo0[3], hi0[3];
  float lo1[3], hi1[3];
  int32_t child0, child1, count0, count1;
};
static_assert(sizeof(Node) == 64, "node layout");

// Triangle in BVH order, 48 bytes: first vertex, two edges, primitive id.
struct alignas(16) Tri {
  float p0[3]; int32_t prim;
  float e1[3]; float pad1;
  float e2[3]; float pad2;
};
static_assert(sizeof(Tri) == 48, "tri layout");

// Naive-AD tape: one record per (vertex, path), vertex-major [D][N].
// flags bits: 0..26 texel index, 27 lambert, 28 valid connection,
// 29 scattered (beta_{j+1} = beta_j * rho_j), 30 dielectric.
struct alignas(16) TapeRec {
  uint32_t tf;
  float g;           // connection factor: C_j = beta_j * rho_j * g
  float ux, uy;      // film position u_j
  float b[3];        // beta_j, throughput arriving at x_j
  float pad;
};
static_assert(sizeof(TapeRec) == 32, "tape layout");
constexpr uint32_t kTexMask = (1u << 27) - 1u;
constexpr uint32_t kTfLambert = 1u << 27, kTfValid = 1u << 28, kTfScatter = 1u << 29,
                   kTfDielectric = 1u << 30, kTfConductor = 1u << 31;

// ResLRB per-path record (Sec. 4.2.1): selected depth R (0 = none), weight
// Omega_k/omega_R, film position u_R and the reweighted splat S_hat.
struct alignas(16) ResRec {
  int32_t R; float W;
  float ux, uy;
  float S[3];
  float pad;
};
static_assert(sizeof(ResRec) == 32, "reservoir record layout");

// Buffered two-pass (lrb_2pass) side state: a header per path (the depth of
// its last sensor connection, one bit per vertex for a valid connection) and
// a splat record per (vertex, path), vertex-major [D][N], preallocated for
// every vertex up to the maximum depth and written where a connection is
// valid: the film position u_i and the contribution C_i.
struct alignas(16) SplatHdr {
  int32_t klast;
  int32_t pad;
  uint64_t vmask;
};
static_assert(sizeof(SplatHdr) == 16, "splat header layout");
struct SplatRec {
  float ux, uy;
  float C[3];
};
static_assert(sizeof(SplatRec) == 20, "splat record layout");

// Attached naive-AD tape record, [D][N] x 128 bytes: the detached fields,
// the chart of x_s (triangle slot, v_s), and once x_{s+1} is known the two
// non-trivial rows of J_s = dp_{s+1}/dp_s and dv_{s+1}/d(channels).
struct alignas(16) TapeRecAtt {
  uint32_t tf;
  int32_t slot;
  float v0, v1;
  float g, ux, uy;
  float b[3];
  float J[8];
  float dch[10];
  float pad[2];
};
static_assert(sizeof(TapeRecAtt) == 128, "attached tape layout");

// Attached ResLRB record (Sec. 4.2.2): the detached record plus the chart of
// x_R, beta_R * rho_R and the accumulated Jacobian M_R = J_{R-1}...J_1.
struct alignas(16) ResRecAtt {
  ResRec base;
  int32_t slot;
  float v0, v1;
  float br[3];
  int32_t slot_p;       // chart of x_{R-1} (slot -1: the emitter), for a conductor at x_R
  float vp0, vp1;
  float gw[4];          // sum over the rough-conductor scatters before R of d log w_s / d p_s M_s
  float M[16];
  float pad[3];
};
static_assert(sizeof(ResRecAtt) == 160, "attached reservoir record layout");

// LRB-3 hand-off between the two replays (Sec. 4.3: the per-sample state of
// the method), one entry per path that has something to back-propagate,
// appended by the pass-2 kernel to the region of the path's class (p mod 8;
// eight regions of ceil(N / 8) entries, eight append counters) and read by
// the pass-3 kernel: the path, the depth of its last connection, one bit per
// vertex for a valid connection and delta_total (FP64, Eq. 14); attached
// also A = sum_i a_i M_i (Eq. 18).
struct alignas(8) Lrb3Hand {
  uint32_t path;
  int32_t klast;
  uint64_t vmask;
  double d[3];
};
static_assert(sizeof(Lrb3Hand) == 40, "hand-off layout");
struct alignas(16) Lrb3HandAtt {
  uint32_t path;
  int32_t klast;
  uint64_t vmask;
  double d[3];
  float A[4];
  float pad[2];
};
static_assert(sizeof(Lrb3HandAtt) == 64, "attached hand-off layout");

// float4 slots of one diffuse guide-table entry (8 lobes x 2)
constexpr int kGTabF4 = 16;

struct DevScene {
  const Node* nodes;
  const Tri* tris;
  const int32_t* prim_mat;   // [n_prims]
  const float* prim_uv;      // [n_static][6]
  const int32_t* mat_type;
  const int32_t* mat_tex;
  const float* mat_ior;
  int32_t n_nodes, n_tris, n_static;
  int32_t hf_G; float hf_x0, hf_z0, hf_dx, hf_base; int32_t hf_mat;
  const float* hf_hb;       // [2] least and greatest height (device), refreshed with the heights
  int32_t n_tex, tex_res;
  int32_t em_type;          // 0 area quad, 1 point, 2 directional quad
  int32_t em_tex_res;       // > 0: L_e is an em_tex_res^2 RGB texture over the quad
  float em_o[3], em_e1[3], em_e2[3], em_n[3], em_area;
  float cpos[3], cf[3], cr[3], cu[3];
  float tan_half, aspect, film_area;
  int32_t W, H;
  int32_t stack_n;  // traversal stack entries per lane (BVH depth + 2)
  // guide input normalisation: scene box centre and inverse half extent
  // (static triangles, heightfield footprint at its base, emitter corners)
  float gb_c[3], gb_ih[3];
};

}  // namespace lt
