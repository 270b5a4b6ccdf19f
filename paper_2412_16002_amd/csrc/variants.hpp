// Launchers of the templated kernels, one table per compiled variant
// (dimension, degree, space, system, precision).
#pragma once

#include "coop.hpp"
#include "device.hpp"

namespace crkdg {

// grid workgroups of `threads` threads
using Launch = void (*)(const KArgs&, int grid, int threads, hipStream_t);

struct VariantOps {
  int dim, k, space, system, precision;
  int M, V, NQ, NS;
  int rec_bytes;   // bytes of one deferred-limiter queue record
  int walls;       // reflective and Dirichlet sides built in
  int alpha_modes; // per-point and global Lax-Friedrichs alpha built in
  Launch stage_local, stage_final, limit, cfl, project, queue_local, queue_final;
  Launch stage_local_p, stage_final_p;   // persistent-grid forms
  Launch stage_inner_dg, stage_inner_dg_p; // inner stage with F (standard RKDG)
  // cooperative stage kernels (tensor spaces): one workgroup of 64 V threads
  // per tile of coop_tile[0] x [1] x [2] cells; coop = 0 when not built
  int coop;
  int coop_tile[3];
  Launch coop_local, coop_inner_dg, coop_final;
  Launch coop_inner_dg_bd, coop_final_bd;   // forms with time-dependent boundary data
};

template <int D, int K, int SP, int SYS, typename T> struct Ops {
  using C = Cell<D, K, SP, SYS, T>;
  static void stage_local(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_stage_local<D, K, SP, SYS, T>), dim3(nb), dim3(nt), 0, s, a);
  }
  static void stage_final(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_stage_final<D, K, SP, SYS, T>), dim3(nb), dim3(nt), 0, s, a);
  }
  static void stage_local_p(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_stage_local_p<D, K, SP, SYS, T>), dim3(nb), dim3(nt), 0, s, a);
  }
  static void stage_final_p(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_stage_final_p<D, K, SP, SYS, T>), dim3(nb), dim3(nt), 0, s, a);
  }
  static void stage_inner_dg(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_stage_inner_dg<D, K, SP, SYS, T>), dim3(nb), dim3(nt), 0, s, a);
  }
  static void stage_inner_dg_p(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_stage_inner_dg_p<D, K, SP, SYS, T>), dim3(nb), dim3(nt), 0, s, a);
  }
  static void limit(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_limit<D, K, SP, SYS, T>), dim3(nb), dim3(nt), 0, s, a);
  }
  static void cfl(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_cfl<D, K, SP, SYS, T>), dim3(nb), dim3(nt), 0, s, a);
  }
  static void project(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_project<D, K, SP, SYS, T>), dim3(nb), dim3(nt), 0, s, a);
  }
  static void queue_local(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_limit_queue<D, K, SP, SYS, T, false>), dim3(nb), dim3(nt), 0, s, a);
  }
  static void queue_final(const KArgs& a, int nb, int nt, hipStream_t s) {
    hipLaunchKernelGGL((k_limit_queue<D, K, SP, SYS, T, true>), dim3(nb), dim3(nt), 0, s, a);
  }
  static VariantOps make() {
    return VariantOps{D, K, SP, SYS, sizeof(T) == 8 ? CRKDG_FP64 : CRKDG_MIXED,
                      C::M, C::V, C::S::NQ, C::NS, static_cast<int>(sizeof(typename C::Record)), C::WALLS ? 1 : 0,
                      C::ALPHA_MODES ? 1 : 0,
                      &stage_local, &stage_final, &limit, &cfl, &project, &queue_local, &queue_final,
                      &stage_local_p, &stage_final_p, &stage_inner_dg, &stage_inner_dg_p,
                      0, {0, 0, 0}, nullptr, nullptr, nullptr, nullptr, nullptr};
  }
};

// A variant whose stage kernels are the cooperative ones (tensor spaces in 2D
// and 3D, and P^k inside Q^k): every boundary kind and alpha mode is built
// in; the limiter, wave-speed, projection and queue kernels stay the
// one-thread-per-cell ones of the stored space.
template <int D, int K, int SYS, typename T, int TX, int TY, int TZ, int SP = SP_Q> struct OpsCoop {
  using B = Ops<D, K, SP, SYS, T>;
  static constexpr int NT = 64 * Phys<D, SYS>::V;
  static void local(const KArgs& a, int nb, int, hipStream_t s) {
    hipLaunchKernelGGL((k_coop_stage<D, K, SP, SYS, T, TX, TY, TZ, 0>), dim3(nb), dim3(NT), 0, s, a);
  }
  static void inner_dg(const KArgs& a, int nb, int, hipStream_t s) {
    hipLaunchKernelGGL((k_coop_stage<D, K, SP, SYS, T, TX, TY, TZ, 1>), dim3(nb), dim3(NT), 0, s, a);
  }
  static void final_(const KArgs& a, int nb, int, hipStream_t s) {
    hipLaunchKernelGGL((k_coop_stage<D, K, SP, SYS, T, TX, TY, TZ, 2>), dim3(nb), dim3(NT), 0, s, a);
  }
  static void inner_dg_bd(const KArgs& a, int nb, int, hipStream_t s) {
    hipLaunchKernelGGL((k_coop_stage<D, K, SP, SYS, T, TX, TY, TZ, 1, true>), dim3(nb), dim3(NT), 0, s, a);
  }
  static void final_bd(const KArgs& a, int nb, int, hipStream_t s) {
    hipLaunchKernelGGL((k_coop_stage<D, K, SP, SYS, T, TX, TY, TZ, 2, true>), dim3(nb), dim3(NT), 0, s, a);
  }
  static VariantOps make() {
    using C = Cell<D, K, SP, SYS, T>;
    return VariantOps{D, K, SP, SYS, sizeof(T) == 8 ? CRKDG_FP64 : CRKDG_MIXED,
                      C::M, C::V, C::S::NQ, C::NS, static_cast<int>(sizeof(typename C::Record)), 1, 1,
                      nullptr, nullptr, &B::limit, &B::cfl, &B::project, &B::queue_local, &B::queue_final,
                      nullptr, nullptr, nullptr, nullptr,
                      NT, {TX, TY, TZ}, &local, &inner_dg, &final_, &inner_dg_bd, &final_bd};
  }
};

// per-translation-unit registries (defined in variants_*.hip)
int variants_v1d(const VariantOps** out);
int variants_v2d_q_adv(const VariantOps** out);
int variants_v2d_p_adv(const VariantOps** out);
int variants_v2d_q12_euler(const VariantOps** out);
int variants_v2d_q3_euler(const VariantOps** out);
int variants_v2d_p_euler(const VariantOps** out);
int variants_v3d_q1(const VariantOps** out);
int variants_v3d_q2_adv(const VariantOps** out);
int variants_v3d_q2_euler(const VariantOps** out);
int variants_v3d_p(const VariantOps** out);
int variants_v3d_p2_euler(const VariantOps** out);
int variants_v3d_p3_euler(const VariantOps** out);
int variants_v3d_q3_euler(const VariantOps** out);
int variants_v3d_k3_adv(const VariantOps** out);
int variants_swe_1d_q(const VariantOps** out);
int variants_swe_2d_p(const VariantOps** out);

}  // namespace crkdg
