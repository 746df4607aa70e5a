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
  float emit_factor;    // beta_0 = L_e * emit_factor
  int32_t n_texels;     // n_tex * tex_res^2
  const uint8_t* mask;
  uint32_t* sig;
  uint32_t* info;
  const float* albedo;
  const float* Le;
  const float* heights;
  unsigned int* counter;
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
  float* g_heights;
  unsigned long long* stats;  // [0] guard triggers, [1] non-finite drops
  int32_t hgrad_lds;          // heights gradients accumulated per workgroup in LDS
};

hipError_t launch_trace(const PassArgs& A, bool tape, bool resv, int grid, int block, hipStream_t s);
hipError_t launch_naive_bwd(const PassArgs& A, int grid, hipStream_t s);
hipError_t launch_reslrb_bwd(const PassArgs& A, int grid, int block, hipStream_t s);
hipError_t launch_lrb3_bwd(const PassArgs& A, int grid, int block, hipStream_t s);
hipError_t launch_lrb3_att(const PassArgs& A, int grid, hipStream_t s);
hipError_t launch_trace_att(const PassArgs& A, bool tape, bool resv, int grid, hipStream_t s);
hipError_t launch_naive_att_bwd(const PassArgs& A, int grid, hipStream_t s);
hipError_t launch_reslrb_att(const PassArgs& A, int grid, hipStream_t s);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s);
hipError_t launch_fill_u32(unsigned int* p, size_t n, unsigned int v, hipStream_t s);
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s);
hipError_t launch_add_le(const double* acc, float* dst, hipStream_t s);
hipError_t launch_loss(const float* I, const float* T, size_t n, float* dI, double* acc, float* loss,
                       hipStream_t s);
hipError_t launch_hf_tris(const DevScene& sc, const int32_t* slot_of_prim, Tri* tris, const float* h,
                          hipStream_t s);
hipError_t set_lds_limit(int bytes);
hipError_t read_counters(uint64_t* out, bool reset, hipStream_t s);
hipError_t launch_refit_level(Node* nodes, const Tri* tris, const int32_t* level_nodes, int n, hipStream_t s);

}  // namespace lt
