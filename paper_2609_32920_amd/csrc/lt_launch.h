// Kernel argument block and launchers (host side of lt_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "lt_common.h"

namespace lt {

struct PassArgs {
  DevScene sc;
  uint64_t seed;
  int32_t n_paths;
  int32_t D;
  uint32_t flags;
  float Kfilm;          // width*height / (A_film * N)
  int32_t n_texels;     // n_tex * tex_res^2
  const uint8_t* mask;
  uint32_t* sig;
  uint32_t* info;
  const float* albedo;
  const float* Le;
  const float* heights;
  const float* nmap;          // normal-map slopes [G][G][2] of the heightfield, or null
  unsigned int* counter;      // work counters (a block of kCtrBlock u32, zero at launch)
  // forward outputs
  float* image;
  TapeRec* tape;
  int32_t* tape_len;
  ResRec* res;
  // attached side state (forward writes, backward reads)
  TapeRecAtt* tape_att;
  float* emit_d;         // [N][2] dv_1 / dH_1 of the emitted ray
  ResRecAtt* res_att;
  const ResRecAtt* res_att_in;
  // backward inputs / outputs
  const float* dI;
  const TapeRec* tape_in;
  const int32_t* tape_len_in;
  const ResRec* res_in;
  float* g_albedo;
  double* g_Le_acc;
  float* g_le_tex;            // textured emitter: the caller's [R][R][3] gradient, or null
  float* g_heights;
  float* g_nmap;              // normal-map gradients [G][G][2], or null
  unsigned long long* stats;  // [0] guard triggers, [1] non-finite drops
  int32_t hgrad_lds;          // heights gradients accumulated per workgroup in LDS
  int32_t agrad_lds;          // albedo gradients accumulated per workgroup in LDS
  int32_t legrad_lds;         // textured-emitter gradients accumulated per workgroup in LDS (past the albedo copy)
  const float4* guide_rec;    // guided emission (direction, density) per path, or null
  const float4* gtab;         // diffuse guide table [2 n_texels][16], or null (cosine scatter)
  int32_t cond;               // the scene has rough conductors: attached kernels carry their terms
  float* tape_gw;             // naive tape with a diffuse guide: scatter weight [D][n_paths]
  const float* tape_gw_in;
  float* gsamp;               // diffuse guide training samples [n_paths][12], or null
  float* contrib;             // per-path image contribution sum_i lum(C_i), or null
  // LRB-3 as two kernels: pass 2 appends a hand-off entry per path with a
  // connection, pass 3 replays the appended paths
  SplatHdr* spl_hdr;          // buffered two-pass: per-path header [n_paths] (forward writes)
  SplatRec* spl;              // and splat records [D][n_paths]
  const SplatHdr* spl_hdr_in; // (backward reads)
  const SplatRec* spl_in;
  Lrb3Hand* hand;             // detached entries [8][hand_region]
  Lrb3HandAtt* hand_att;      // attached entries [8][hand_region]
  uint32_t hand_region;       // entries per class region, ceil(n_paths / 8)
  unsigned int* hand_app;     // pass 2's append counter of each class (a block of kCtrBlock u32)
  unsigned int* counter3;     // pass 3's work counters (a block of kCtrBlock u32)
  // camera side (k_camera, k_camera_prb): flags bit 0 = every sample, not only
  // those whose first vertex is specular; each sample weighs W*H / N
  float spp_inv;
};

typedef unsigned int lt_u32x4 __attribute__((ext_vector_type(4)));

// Emission-guide passes.
struct GuideArgs {
  DevScene sc;
  uint64_t seed;
  const uint64_t* seed_ptr;  // emit: seed read from device memory when set (graph replays)
  int64_t count;             // paths (emit) or samples (grad) or items (eval)
  const float* w;            // FP32 parameters (biases read from here)
  const lt_u32x4* packed;    // bf16 operand tiles from k_guide_pack
  float4* rec;               // emit: per-path (direction, density)
  float* samples;            // emit: optional [count][12] out; grad: [count][12] in
  const float* contrib;      // emit: per-path S for the samples, or null
  const float* x;            // eval inputs [count][3]
  const float* n;
  float* out;                // eval outputs [count][41]
  float* partial;            // grad: [grid][11435] partial sums (gradient, loss, Z)
  float4* table;             // table: [count][16] guide-table entries out
};

size_t guide_packed_bytes();
size_t guide_partial_floats();
hipError_t guide_init();
hipError_t launch_guide_pack(const float* w, void* packed, hipStream_t s);
hipError_t launch_guide_eval(const GuideArgs& G, int grid, hipStream_t s);
hipError_t launch_guide_emit(const GuideArgs& G, int grid, hipStream_t s);
// diffuse guide table: count = 2 x texels, x / n the texel centres and normals
hipError_t launch_guide_table(const GuideArgs& G, int grid, hipStream_t s);
hipError_t launch_guide_grad(const GuideArgs& G, int grid, hipStream_t s);
hipError_t launch_guide_reduce(const float* partial, int n_part, float* grad, float* loss, hipStream_t s);
hipError_t launch_guide_adam(float* w, const float* grad, float* m, float* v, int n, float lr, float b1, float b2,
                             float eps, float c1, float c2, hipStream_t s);

hipError_t launch_trace(const PassArgs& A, bool tape, bool resv, int grid, int block, hipStream_t s);
// forward that also writes the buffered two-pass splat records
hipError_t launch_trace_splats(const PassArgs& A, bool resv, int grid, int block, hipStream_t s);
// forward that also writes each path's diffuse-guide training sample (A.gsamp)
hipError_t launch_trace_gsamples(const PassArgs& A, int grid, int block, hipStream_t s);
// buffered two-pass backward: delta_total from the records, one replay
hipError_t launch_lrb2_bwd(const PassArgs& A, int grid, int block, hipStream_t s);
// batches: `table` is a DEVICE array of n PassArgs; stack_n the largest
// traversal stack among them
hipError_t launch_trace_batch(const PassArgs* table, int n, int stack_n, int grid, int block, hipStream_t s);
// one table entry's forward (the table pointer already offset to it)
hipError_t launch_trace_entry(const PassArgs* entry, bool hf, int stack_n, int grid, int block, hipStream_t s);
// grad_lds: LDS bytes past the traversal stacks for per-workgroup gradient
// copies; hf: some entry's scene has a heightfield
hipError_t launch_lrb3_batch(const PassArgs* table, int n, bool hf, int stack_n, size_t grad_lds, int grid, int block,
                             hipStream_t s);
// one detached table entry (the table pointer already offset to it)
hipError_t launch_lrb3_entry(const PassArgs* entry, bool hf, int stack_n, size_t grad_lds, int grid, int block,
                             hipStream_t s);
hipError_t launch_lrb3_att_batch(const PassArgs* table, int n, int stack_n, size_t grad_lds, int grid, hipStream_t s);
// one attached table entry (the table pointer already offset to it)
hipError_t launch_lrb3_att_entry(const PassArgs* entry, int stack_n, size_t grad_lds, int grid, int block,
                                 hipStream_t s);
// the same entry through the two-kernel LRB-3 (pass 2 at 256 threads, pass 3
// at block3 with grad_lds past its stacks)
hipError_t launch_lrb3_att_split_entry(const PassArgs* entry, int stack_n, size_t grad_lds, int grid2, int grid3,
                                      int block3, hipStream_t s);
hipError_t launch_naive_bwd(const PassArgs& A, int grid, hipStream_t s);
hipError_t launch_reslrb_bwd(const PassArgs& A, int grid, int block, hipStream_t s);
hipError_t launch_lrb3_bwd(const PassArgs& A, int grid, int block, hipStream_t s);
// LRB-3 as two kernels with the per-path hand-off of Lrb3Hand / Lrb3HandAtt
hipError_t launch_lrb3_p2(const PassArgs& A, int grid, int block, hipStream_t s);
hipError_t launch_lrb3_p3(const PassArgs& A, int grid, int block, hipStream_t s);
hipError_t launch_lrb3_att_p2(const PassArgs& A, int grid, int block, hipStream_t s);
hipError_t launch_lrb3_att_p3(const PassArgs& A, int grid, int block, hipStream_t s);
hipError_t launch_lrb3_att(const PassArgs& A, int grid, int block, hipStream_t s);
hipError_t launch_trace_att(const PassArgs& A, bool tape, bool resv, int grid, hipStream_t s);
hipError_t launch_naive_att_bwd(const PassArgs& A, int grid, hipStream_t s);
hipError_t launch_reslrb_att(const PassArgs& A, int grid, int block, hipStream_t s);
// camera side of the bidirectional combination: forward (adds to A.image)
// and the path-replay backward (A.dI in, albedo / emitter gradients out)
hipError_t launch_camera(const PassArgs& A, int grid, int block, hipStream_t s);
hipError_t launch_camera_prb(const PassArgs& A, int grid, int block, hipStream_t s);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s);
hipError_t launch_fill_u32(unsigned int* p, size_t n, unsigned int v, hipStream_t s);
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s);
hipError_t launch_add_le(const double* acc, float* dst, hipStream_t s);
hipError_t launch_loss(const float* I, const float* T, size_t n, float* dI, double* acc, float* loss,
                       hipStream_t s);
// heightfield triangles from the heights (slots n_static...) and the
// heights' least and greatest value into hb[2]
hipError_t launch_hf_tris(const DevScene& sc, Tri* tris, const float* h, float* hb, hipStream_t s);
hipError_t set_lds_limit(int bytes);
// Workgroups of a backward kernel resident per CU at `block` threads and
// `lds` dynamic LDS bytes (0 if it cannot launch or the query fails).
enum class BwdKernel { naive, reslrb, lrb3, naive_att, reslrb_att, lrb3_att, lrb3_batch, lrb3_att_batch, lrb3_att_entry,
                       lrb3_p2, lrb3_p3, lrb3_att_p2, lrb3_att_p3, lrb2, lrb3_att_p3_entry, camera_prb, lrb3_entry,
                       lrb3_att_p3_cond, lrb3_att_cond };
int resident_groups(BwdKernel k, int block, size_t lds);
hipError_t read_counters(uint64_t* out, bool reset, hipStream_t s);

}  // namespace lt
