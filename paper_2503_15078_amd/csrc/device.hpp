// Device data layout and kernel entry points of the gfx950 solver.
//
// All node arrays are structure-of-arrays float32 in the internal (nested-dissection
// postorder) numbering, padded to N4 = round_up(N, 4) + 4 entries per coordinate so
// that the S pass can read b in aligned float4 groups.  A batch of scenes is the
// concatenation of its scenes' node ranges: the block-diagonal system has one
// elimination forest, so the element, S and S^T kernels do not know about scenes.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lg {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kMaxObstacles = 64;
constexpr int kDelTile = 16;      // Delassus tile (contacts x contacts)
// Row stride of a scene's Delassus block: its contact count rounded up to 4 (rows are
// 16-byte aligned; the pad entries are zero).
__host__ __device__ inline int kstride(int cnt) { return (cnt + 3) & ~3; }
constexpr int kDelChunk = 256;    // Delassus depth chunk staged in LDS
constexpr int kMaxGroup = 8;      // S-pass rows / S^T-pass columns per wavefront, at most
constexpr int kMaxCrIters = 1024;
constexpr int kMlpParams = 20752;   // 16x128 + 128 + 128x128 + 128 + 16x128 + 16 (padded shapes)
constexpr int kMlpMaxBlocks = 256;  // blocks of one training launch (64 samples each)
constexpr int kMlpMaxBatch = 64 * kMlpMaxBlocks;
constexpr int kCrMaxBlocks = 256;   // blocks of the CR launch, at most one per CU
// arrival flags of the CR launch's device-wide barriers: two slots (barrier parity) of one
// flag per block, each flag on its own 128-byte line
constexpr int kCrFlagStride = 32;
constexpr int kCrSyncWords = 2 * kCrMaxBlocks * kCrFlagStride;
// scenes of one handle: a CR block keeps a slot per scene between its first and last
// contact (empty scenes included), in LDS tables of this many entries
constexpr int kMaxScenes = 256;
constexpr int kCrMaxBarriers = 2 * kMaxCrIters + 2;  // device-wide barriers of one CR launch

struct ObstacleDev {
  int type;
  int scene;
  double geom[10];
  double mu;
  double vel[3];
};

// Pointers to device memory, passed by value to kernels.
struct Dev {
  // sizes
  int N, N4, M, P, G, NS;          // nodes, padded nodes, tets, pins, pin groups, scenes
  int CMAX;                        // contact capacity (all scenes)
  int64_t KCAP;                    // Delassus storage capacity (floats)
  int nseg, nlong;                 // S-pass segments, multi-segment rows
  int elem_block;                  // threads per block of the element kernel (64..256)
  double h;
  double g[3];
  int cr_iters;
  int warm;
  int ncp, precond;                // SIM_NCP_*, SIM_PRECOND_*
  int global_step;                 // SIM_GLOBAL_*
  int lg_form;                     // SIM_LG_* (1: ADMM-PD duals in the local step)
  // nodes
  float *qt, *vt, *qp, *q, *b, *y, *tgt, *pin_w, *tmp;
  int *node_scene;
  int *iperm_caller;               // internal node -> caller node
  int *g_ptr, *g_slot;             // node -> corner-force offsets (3 corner M + tet) gather lists
  // pins
  int *pin_node, *pin_group;
  double *pin_x0;                  // [3][P]
  double *grp;                     // [G][9]: lin(3), ang(3), pivot(3)
  // tets
  int *tidx;                       // [4][M]
  float *dinv;                     // [9][M] rows d1,d2,d3
  float *hw, *tmu, *tlam, *tk;     // h^2 w, mu, lambda, k
  unsigned char *tmodel;
  float *fc;                       // [12][M] corner forces
  float *dual;                     // [9][M] ADMM-PD dual variables (row-major 3x3 per tet)
  // S storage
  int64_t *row_ptr;
  int *row_lo4;
  float *row_val;
  int row_group, col_group;        // group size limits of the S and S^T passes (1, 2, 4, 8)
  // S-pass segments: a group of up to row_group consecutive rows stored from the same
  // column quad, cut along its columns; seg_row = first row (-(row + 1) if the group has
  // several segments), seg_q0 = first quad of the segment, seg_len = its floats per row,
  // seg_off = row_ptr of the first row + 4 seg_q0, seg_col0 = its first column
  int *seg_row, *seg_ng, *seg_q0, *seg_len, *seg_col0;
  int64_t *seg_off;
  int *long_row, *long_seg0, *long_nseg, *long_ng;
  float *partial;                  // [3][row_group][nseg]
  int64_t *col_ptr;
  float *col_val;
  int64_t *colp_ptr;               // [N+1] S^T-pass copy of the columns (multiples of 4)
  float *colp_val;                 // runs stored from node a & ~3, zero outside the run
  int *run_ptr;                    // [N+1] chain runs of each column's ancestor path
  int *run_a, *run_e;              // first and last node of each run
  int n_stgrp;                     // S^T-pass groups: up to col_group consecutive columns
  int *stgrp_j0, *stgrp_ng;        // of one chain (first column, count)
  int *parent, *lo, *depth, *chain_end;
  int *frange;                     // [2][N] per-row contact range of the frame
  // scenes
  int *scene_node0;                // [NS+1]
  int *scene_obst0;                // [NS+1]
  double *scene_margin;            // [NS]
  ObstacleDev *obst;               // [kMaxObstacles * NS] (flat, scene ranges)
  // contacts (internal order: by internal node, then obstacle)
  int *n_contacts;                 // [1]
  int *overflow;                   // [1]
  int *cnt, *blk;                  // collision scan scratch [N], [N/256+1]
  int *c_node, *c_obst, *c_scene;
  float *cC;                       // [9][CMAX] frame rows n, f1, f2
  double *cC64, *c_dn64;           // the same frame and d_n in float64 (normal gap)
  float *c_dn, *c_df, *c_mu, *c_rn, *c_rf;  // df: [2][CMAX]
  double *c_gap;
  float *lam;                      // [3][CMAX]
  int *cs_off;                     // [NS+1] contact range per scene
  int64_t *k_off;                  // [NS+1] Delassus block offsets
  int *tile_off;                   // [NS+1] Delassus tile offsets
  float *K;
  int *ad;                         // adjacent LCA depth [CMAX]
  // previous frame
  int *pc_count;
  int *pc_node, *pc_obst;
  float *pc_world;                 // [3][CMAX]
  // iteration scratch [3][CMAX] each
  float *Om, *Et, *hv, *X, *F;     // hv: h_vec - Omega H u (delta form)
  float *cr_Z;                     // [2][2][3][CMAX] exchanged C^T (Omega v) of the CR launch
  float *cr_prod;                  // per-(block, scene slot) partial sums of the CR launch
  unsigned *cr_sync;               // [kCrSyncWords] barrier arrival flags of the CR launch
  unsigned long long *cr_clock;    // null, or [2 + 4 kCrMaxBarriers] wall-clock stamps of CR block 0
  float cr_tol;                    // relative CR residual tolerance (0: fixed count)
  // learned warm start
  double *ell;                     // [NS] mean rest edge length per scene
  float *c_feat;                   // [CMAX][16] features of the frame's contacts
  float *c_comp;                   // [CMAX] compliance e of bilateral (binding) rows, -1: unilateral
  float *inv_mass;                 // [N] 1 / lumped mass (mass-inverse preconditioner)
  int *a_ptr, *a_idx;              // A_n in internal order (CSR) for the Jacobi global step
  float *a_val, *a_dinv;           // its values and 1 / diagonal
  float *mlp_P;                    // [kMlpParams] network parameters (float32 master copy)
  float *lam_ml;                   // [3][CMAX] learned candidate of the frame's start impulses
  float *wl;                       // [6][CMAX] world impulses C^T lambda of the plain, learned start
  float *judge;                    // [2][NS] linearized NCP residual of the plain, learned start
  // self contact (single-scene handles): vertex-triangle rows with four entries each,
  // stored after the obstacle contacts, which keep their node order
  int self_on;
  int T, NSV;                      // surface triangles, surface vertices
  int *tri_v;                      // [3][T] corners (internal ids), normal outward
  int *sv;                         // [NSV] surface vertices (internal ids) by caller id
  int *vt_ptr, *vt_idx;            // [NSV+1] incident triangles of each surface vertex, ascending
  double *tri_n;                   // [2][3][T] unit normals at q_t and q~ (per frame)
  int *sv_cnt;                     // [NSV] self contacts per surface vertex, then offsets
  float self_mu;
  int *n_obst_c;                   // [1] contacts from obstacles (the first rows)
  int *ent_node;                   // [4][CMAX] entries of the self rows (internal ids)
  double *ent_w;                   // [4][CMAX] their signs (1, -w_a, -w_b, -w_c)
  int *se_node, *se_row;           // [4 CMAX] self entries sorted by (node, row, corner)
  float *se_w;                     // their signs
  int *se_count;                   // [1]
  int *frange2;                    // [2][N] per-row range of the sorted self entries
  // frames iterated to tolerance: the iterations run in chunks replayed without a host
  // round trip; done[0] is set once the frame has converged (or hit max_iters, or failed)
  // and every iteration kernel then returns at once.  Null outside such frames.
  int *done;                       // [1]
  int *iter_count;                 // [1] iterations run in the current frame
  float ncp_tol;                   // NCP residual tolerance (metres)
  int max_iters;                   // iteration cap of such frames
  // frame state
  double *t;                       // [1] simulation time at frame start
  float *res;                      // [NS] NCP residual per scene
  int *bad;                        // [0] frame invalid (non-finite state or [1]); [1] CR barrier abandoned
};

// End of the single-node (obstacle) contacts of scene s: self-contact rows follow them.
__device__ inline int obst_end(const Dev& d, int s) {
  return d.self_on ? min(d.n_obst_c[0], d.cs_off[s + 1]) : d.cs_off[s + 1];
}

// True in a frame iterated to tolerance once it has converged (uniform across the grid).
__device__ inline bool frame_done(const Dev& d) {
  return d.done != nullptr && __builtin_amdgcn_readfirstlane(*d.done) != 0;
}

// kernels (launch helpers live in the .hip files)
void launch_predict(const Dev& d, hipStream_t st);
void launch_pins(const Dev& d, hipStream_t st);
void launch_collide(const Dev& d, hipStream_t st);
void launch_self_entries(const Dev& d, hipStream_t st);
void launch_frames_for_list(const Dev& d, hipStream_t st);
void launch_delassus(const Dev& d, hipStream_t st);
void launch_warm_start(const Dev& d, hipStream_t st, int keep_lambda);
void launch_element(const Dev& d, hipStream_t st);
void launch_zero_dual(const Dev& d, hipStream_t st);
void launch_gather(const Dev& d, hipStream_t st);
void launch_spmv_S(const Dev& d, hipStream_t st, const float* b, float* y);
void launch_spmv_St(const Dev& d, hipStream_t st, const float* y, const float* base, float* u);
void launch_contact_prep(const Dev& d, hipStream_t st);
void launch_mlp_forward(const float* P, const float* X, float* Y, int n, hipStream_t st);
int mlp_train_blocks(int n);
void launch_mlp_train(const float* P, const float* X, const float* T, int n, float* partial, hipStream_t st);
void launch_mlp_adam(float* P, float* M, float* V, const float* partial, int n, float lr, float b1, float b2,
                     float eps, float c1, float c2, int update, float* grad_out, float* loss_out, hipStream_t st);
void launch_mlp_features(const Dev& d, hipStream_t st);
void launch_mlp_warm(const Dev& d, hipStream_t st);
void launch_warm_judge(const Dev& d, hipStream_t st);
void launch_mlp_targets(const Dev& d, float* out, hipStream_t st);
hipError_t launch_cr(const Dev& d, hipStream_t st, int cr_blocks, int variant);  // variant: SIM_CR_*
void launch_zero_cr_sync(const Dev& d, hipStream_t st);
void launch_apply_forces(const Dev& d, hipStream_t st);
void launch_jacobi_global(const Dev& d, hipStream_t st);
int lg_energy_blocks(const Dev& d);
void launch_lg_energy(const Dev& d, hipStream_t st, double* part);
void launch_force_ranges(const Dev& d, hipStream_t st);
void launch_residual(const Dev& d, hipStream_t st);
void launch_reset_convergence(const Dev& d, hipStream_t st);
void launch_convergence_check(const Dev& d, hipStream_t st);
void launch_integrate(const Dev& d, hipStream_t st);
void launch_check_finite(const Dev& d, hipStream_t st);
void launch_export_positions(const Dev& d, hipStream_t st, float* out);
int cr_max_blocks();
int64_t cr_partial_floats(int blocks, int scenes);

}  // namespace lg
