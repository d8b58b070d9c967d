// Device-side data layout shared by the kernels and the host launcher.
//
// Every per-vertex quantity is structure-of-arrays over the concatenation of
// all environments: component c of vertex i lives at [c * NV + i].  Per-tet
// data is SoA the same way over all tets.  Per-contact data lives in one slab
// of `cap` records per environment.  The explicit inverse Gbar = Abar^-1 of
// each environment is a dense row-major n x ld block (ld = n rounded up to 32,
// so that every row starts on a 128-byte line).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flash {

constexpr int kMaxObs = 4;
constexpr int kMaxGrip = 2;                       // grippers (bilateral attachment) per env
constexpr int kCacheSlots = kMaxObs + kMaxGrip;   // constraint rows per vertex: warm-start cache entries
constexpr int kBlock = 256;
constexpr int kBK = 16;         // panel width of the blocked factorisations in the contact solve
constexpr int kWsMaxFail = 3;   // learned-start failures after which an env keeps the plain start

// Kernel classes for event timing (flash_kernel_name order).
enum KernelId {
  K_DETECT = 0, K_GATHER, K_PROJECT, K_ASSEMBLE, K_APPLY, K_CSP, K_CORRECT, K_FINALIZE,
  K_MLP, K_FUSED, K_COUNT
};

template <class T>
struct DevBatch {
  int n_envs;
  int NV, NT;                 // total vertices / tets (tets: 4-node; tris: 3-node use the same arrays)
  int cap;                    // contact capacity per env
  int rmax;                   // capacity of the Woodbury capacitance system per env (3 rows per contact)
  int rlds;                   // systems of up to rlds rows keep their LU panel in LDS, larger ones in lupan
  int max_newton;
  int lg_iterations;
  double h;
  double g[3];
  double margin;
  double tol;
  double max_force;
  int warm_start;             // FLASH_WS_*
  int reuse;                  // reuse capacitance factorisations across Newton iterations
  int lite;                   // 1: fixed-budget lightweight contact update (inertia-only metric)
  int lite_global;            // 1: the lightweight update runs from global memory (k_lite_update)
  int* lite_done;             // [n_envs] the env's lightweight iteration stopped in this local-global
                              // iteration (tolerance or budget); its position updates are skipped
  unsigned long long* lite_r; // [n_envs x lg_iterations x (max_newton + 1)] residual of each update of
                              // the step (bits of a non-negative double, combined by atomic maximum)

  const int* voff;            // [n_envs+1]
  const int* toff;            // [n_envs+1]
  const int* vert_env;        // [NV]
  const int* tet_env;         // [NT]

  T* x;                       // [3*NV] positions at step start
  T* v;                       // [3*NV]
  T* u;                       // [3*NV] displacement q - x of the current iterate
  T* ut;                      // [3*NV] predicted displacement h v + h^2 g
  T* z;                       // [3*NV] Gbar b
  T* b;                       // [3*NV] right-hand side in displacement form
  const T* mass;              // [NV]

  const int* tet_idx;         // [4*NT] global vertex ids
  const T* tet_B;             // [9*NT] D_m^-1 row-major (B[r][c] at (3r+c)*NT)
  const T* tet_w;             // [NT]
  T* fel;                     // [3 per incidence] vertex forces w (p - F_x) gradN_a, vertex-ordered
  const int* inc_off;         // [NV+1] incidence ranges per vertex (element slots, then hinge slots)
  const int* slot;            // [4*NT] incidence slot of (element t, local vertex a) at t*4+a (-1: none)
  int NH;                     // bending hinges over all envs
  const int* hinge_idx;       // [4*NH] global vertex ids (edge x0 x1, opposite x2 x3)
  const T* hinge_alpha;       // [4*NH] stencil alpha
  const T* hinge_w;           // [NH] weight w_h
  const int* hinge_slot;      // [4*NH] incidence slots

  const T* G;                 // dense inverses
  const int64_t* goff;        // [n_envs] element offset of env block
  const int* gld;             // [n_envs] leading dimension

  // obstacles [n_envs * kMaxObs]
  int* nobs;                  // [n_envs]
  int* obs_kind;
  int* obs_move;
  double* obs_c;              // [*3]
  const double* obs_R;        // [*9]
  const double* obs_size;     // [*3]
  const double* obs_vel;      // [*3]

  // grippers [n_envs * kMaxGrip] and the vertices they hold (bilateral attachment)
  int* ngrip;                 // [n_envs]
  int* grip_grasp;            // grasp on (1) / off (0)
  int* grip_move;             // steps left to move (negative: forever)
  int* grip_held;             // vertices held after the last detection
  double* grip_c;             // [*3] center at the start of the next step
  const double* grip_vel;     // [*3]
  const double* grip_r;       // capture radius
  int* att_g;                 // [NV] gripper holding the vertex, -1: none
  double* att_off;            // [3 per vertex] offset from the gripper center taken at capture

  // contacts [n_envs * cap]
  int* ccount;                // [n_envs]
  int* cvert;                 // local vertex index
  int* cobs;                  // obstacle index; kMaxObs + g for the attachment row of gripper g
  T* cframe;                  // [9 per contact] columns n, t1, t2: frame[3*a + k] = column a, comp k
  double* cframe64;           // the same frames in FP64 (FP32 batches with an FP64 contact solve; else
                              // nullptr, or cframe itself in FP64 batches)
  T* cd0;
  T* cdob;                    // [2 per contact] T^T dobs
  T* cs;                      // residual scale h^2/m_v
  double* clam;               // [3 per contact] multipliers (n, t1, t2), FP64: the residual scale
                              // h^2/m_v maps FP32 rounding of lambda to ~1e-7 m
  T* cforce;                  // [3 per contact] world force F lambda
  void* cyf;                  // [3 per contact] free displacement in the contact frame (solve scratch)
  int* cnew;                  // 1: no warm start available
  double* cd0d;               // FP64 gap (kept for exact reporting)

  // contact-space scratch, in the contact-solve precision (double when csp64, else T)
  int csp64;                  // 1: the contact-space solve runs in FP64
  void* Gc;                   // [cap*cap per env] Gbar restricted to contacts
  void* Ginv;                 // [cap*cap per env] inverse on the base set
  void* Cm;                   // [rmax*rmax per env] capacitance matrix + row data
  int* base;                  // [cap per env] base-set contact ids (ordered)
  void* scr;                  // [cap*16 per env] panel scratch of the blocked inverse
  void* lupan;                // [rmax*(kBK+2) per env] LU panel (row stride kBK+1) and solve vector of
                              // systems above rlds rows
  int* nbase;                 // [n_envs]
  int* lust;                  // [4 per env] stored capacitance factorisation: valid, rows, base version x2

  // warm-start cache [NV * kCacheSlots]
  T* cache_f;                 // [3 per entry] world force
  int* cache_stamp;
  int* stamp;                 // [1] step counter (device side)

  // per env outputs
  double* resid;              // [n_envs]
  double* resid_hist;         // [4 per env] since the last reset: max residual, steps above ncp_tol,
                              // Newton iterations, steps
  double ncp_tol;             // acceptance tolerance of the end-of-step residual
  int* iters;                 // [n_envs] Newton iterations this step
  int* refac;                 // [n_envs]
  int* flags;                 // [n_envs]
  int* fp64_polar;            // [n_envs]
  unsigned long long* phase;  // [n_envs * 12] contact-solve phase ticks and event counts (nullptr: off)

  // scheduling of the per-env contact solves (nullptr: identity order)
  int* order;                 // [n_envs] env of each contact-solve workgroup
  unsigned long long* cost;   // [n_envs] wall-clock ticks of the env's solves since the last ordering

  // learned warm start (optional)
  const double* lam_ml;       // [3 per contact] predicted multipliers (nullptr: off)
  int* ws_state;              // [n_envs] bit 0: this step started from the prediction; bit 2: this
                              // step's solve from the prediction missed the tolerance and restarted;
                              // bits 8-15: such restarts so far; bit 1: prediction disabled after
                              // kWsMaxFail of them
  unsigned long long* ws_hist;  // [2 per env] since the last reset: steps started from the prediction,
                                // steps restarted from the plain start
};

}  // namespace flash
