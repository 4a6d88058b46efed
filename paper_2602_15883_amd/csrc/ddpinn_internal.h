// Internal definitions shared by the HIP kernels and the host runtime of
// libddpinn.  Not part of the public ABI (include/ddpinn.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddp {

constexpr int kWave = 64;
constexpr int kMaxWidth = 256;
constexpr int kMaxWaves = 8;    // waves per workgroup of the network kernels
constexpr int kMaxDepth = 16;
constexpr int kMaxSub = 4096;
constexpr int kSlabChunk = 16;   // slabs summed per thread in the first reduce stage

// Per-subdomain device descriptor (copied into the workspace at create).
struct SubDev {
  const float* theta;
  float* m;
  float* v;
  const float* pde_x;
  const float* obs_x;
  const float* obs_u;
  const float* gh_x;
  const float* gh_up;
  const uint8_t* gh_kind;
  const float* anc_x;
  const float* anc_p;
  float* frag;            // kernel copies of the weights (workspace)
  int32_t n_pde, n_obs, n_gh, n_anc;
  float lam[6];           // effective weights: gh_p^space is 0 on masters
  float inv_n[4];         // 1/n_pde, 1/n_obs, 1/n_gh, 1/n_anc (0 if empty)
  float lo[4], hi[4];
  float cw[4];            // weights of the velocity components in L_obs, L_gh_u
  int32_t is_master;
  int32_t pad_[3];
};

enum : int32_t { ITEM_PDE = 0, ITEM_VALUE = 1 };
enum : int32_t { ITEM_FIRST = 1, ITEM_LAST = 2 };

// One unit of work of the persistent step kernel: a tile of collocation
// points (ITEM_PDE) or of value-only points (observation, ghost, anchor;
// ITEM_VALUE) of one subdomain.
struct Item {
  int32_t sub, kind, start, count;
  int32_t slab;           // gradient slab of the (workgroup, subdomain) segment
  int32_t flags;          // ITEM_FIRST / ITEM_LAST of the segment
  int32_t pad_[2];
};

// Geometry of one network and of the buffers derived from it.  Offsets are
// in floats.
struct Shape {
  int32_t dim, D, W, H, Wp, NW;   // D = dim+1 inputs/outputs; Wp = W padded to 16; NW = Wp/16 row blocks
  int32_t P;                      // packed parameter count
  int32_t act;                    // activation: 0 tanh, 1 sin
  int32_t NWV;                    // waves per workgroup, min(NW, kMaxWaves): wave w owns row
                                  // block w and, when NW > kMaxWaves, row block w + NWV
  int32_t split;                  // two row blocks per wave and the step's LDS plan does not
                                  // fit: one forward activation stack, backward by column halves
  int32_t Kq;                     // ceil(W/4): K-steps of the hidden-layer GEMMs (hidden neurons
                                  // are stored at permuted positions, see hid_pos)
  int32_t pad_;
  // fragment buffer (per subdomain)
  int64_t f_hid;   // hidden layer l (2..H): forward A-fragments at f_hid + (l-2)*2*Wp*Wp,
                   // transposed (backward) A-fragments Wp*Wp further
  int64_t f_w1;    // W1 padded [Wp][D]
  int64_t f_b;     // b_1..b_H padded [H][Wp]
  int64_t f_wo;    // W_{H+1} padded [D][Wp]
  int64_t f_bo;    // b_{H+1} [4]
  int64_t frag_floats;
  // gradient slab (per segment)
  int64_t s_hid;   // dW_l (l = 2..H) in accumulator order at s_hid + (l-2)*Wp*Wp
  int64_t s_b;     // db_1..db_H [H][Wp]
  int64_t s_w1;    // dW_1 [Wp][D]
  int64_t s_wo;    // dW_{H+1} [D][Wp]
  int64_t s_bo;    // db_{H+1} [4]
  int64_t s_loss;  // loss partial sums [8]
  int64_t slab_floats;
  // packed parameter offsets (caller layout)
  int64_t p_w[kMaxDepth + 2];
  int64_t p_b[kMaxDepth + 2];
};

struct StepArgs {
  Shape sh;
  const SubDev* subs;
  const Item* items;
  const int32_t* wg_begin;  // [n_ranges + 1] item ranges
  int32_t* counter;         // next free range (zeroed by prep_kernel); NULL: range = workgroup index
  int32_t n_ranges;
  float* slabs;
  float* stash;
  int64_t stash_per_wg;     // floats
  float nu;
  int32_t lds_floats;
  int32_t prio;             // the younger half of the waves raises its priority for its GEMMs
  int32_t pad_;
};

struct ReduceArgs {
  Shape sh;
  const SubDev* subs;
  const int32_t* seg_begin; // [n_sub + 1] slab range of each subdomain
  const float* slabs;
  float* partial;           // [n_sub][n_chunks][slab_floats] first-stage sums
  int32_t n_chunks;         // ceil(max slabs of one subdomain / kSlabChunk)
  float* loss_out;          // [n_sub][7] or null
  float* grad_out;          // [n_sub][P] or null
  float* loss_ws;           // [n_sub][8] always written (finite check)
  float* gbuf;              // [n_sub][P] gradient
  float* normpart;          // [n_sub][grid blocks] partial sums of g^2
  float* clip_scale;        // [n_sub] min(1, clip / ||g||)
  int32_t n_sub;
  int32_t update;           // run Adam
  int64_t t;                // Adam step (1-based)
  float lr, beta1, beta2, eps;
  float clip;               // global-norm clipping threshold (0: off)
  int32_t pad_;
};

struct PrepArgs {
  Shape sh;
  const SubDev* subs;
  int32_t n_sub;
  int32_t n_counters;
  int32_t* counters;        // range counters of the step launches, zeroed here
};

// Query modes
enum : int32_t { Q_VALUE = 0, Q_UVPW = 1, Q_CHANNELS = 2, Q_RESIDUAL = 3 };

struct QueryArgs {
  Shape sh;
  const SubDev* subs;
  const float* x;           // [n][D]
  float* out;
  const int32_t* perm;      // routed order (null: identity)
  const int32_t* counts;    // [n_sub] points per subdomain (null: single sub)
  const int32_t* offsets;   // [n_sub] start of each subdomain in perm
  int64_t n;
  int32_t sub;              // >= 0: evaluate this subdomain for all points
  int32_t n_sub;
  int32_t what;
  float nu;
  int32_t lds_floats;
  int32_t small;            // one 16-point block per channel (value and gradient modes)
};

struct RouteArgs {
  const float* x;
  int64_t n;
  const float* boxes;       // [n_sub][2][4]
  float gmax[4];
  int32_t n_sub, D, out_cols;
  int32_t* sub_id;          // [n]
  int32_t* counts;          // [n_sub]
  int32_t* cursor;          // [n_sub]
  int32_t* offsets;         // [n_sub + 1]
  int32_t* perm;            // [n]
  float* out;               // NaN rows for points in no box
};

struct ExchangeItem {
  int32_t a, b;             // receiving subdomain, owning neighbour
  int32_t start, count;     // ghost indices of `a` covered by this tile
  int32_t paired;           // neighbour is a master: half the columns evaluate the anchor
  int32_t pad_[3];
};

struct ExchangeArgs {
  Shape sh;
  const SubDev* subs;
  const ExchangeItem* items;
  int32_t n_items;
  int32_t lds_floats;
  float* const* targets;    // [n_sub] device pointers (null for subdomains without faces)
  float x_anc[3];
  int32_t pad_;
};

// Evaluation post-processing: per-snapshot pressure means and error sums.
constexpr int kEvalChunk = 1024;   // points per block in the evaluation kernels
struct EvalArgs {
  const SubDev* subs;
  const float* pred;        // [n][D] routed predictions
  const float* pa;          // [n][D] predictions at (x_anc, t) by the same subdomain
  const float* ref;         // [n][D] reference (u.., p)
  const int32_t* sub_id;    // [n]
  const int64_t* snap_off;  // [n_snap + 1]
  float* mpart;             // [n_snap][nblk][2] sums of processed p and reference p
  float* epart;             // [n_snap][nblk][2 * (D + 1)] error sums
  float* err_out;           // [D + 1]
  int32_t D, n_snap, nblk, pad_;
};

// Routed-query scratch held by the library itself (pinn_query_noalloc): the
// layout of pinn_query's caller scratch for up to kNoallocQueryPoints points
// and kMaxSub subdomains (sub_id and perm [n], counts, cursor and offsets
// [n_sub + 1], each part 256-byte aligned).
constexpr int64_t kNoallocQueryPoints = int64_t(1) << 20;
constexpr size_t kNoallocScratchBytes =
    2 * ((4 * (size_t)kNoallocQueryPoints + 255) & ~size_t(255)) + 3 * ((4 * (size_t)(kMaxSub + 1) + 255) & ~size_t(255));
// device address of the library-held scratch on the current device
hipError_t noalloc_scratch_address(void** ptr);

// Launchers (ddpinn_kernels.hip)
hipError_t launch_prep(const PrepArgs& a, hipStream_t s);
hipError_t launch_step(const StepArgs& a, int tile_points, int n_wg, hipStream_t s);
hipError_t launch_step_timed(const StepArgs& a, int tile_points, int n_wg, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);
hipError_t launch_route(const RouteArgs& a, hipStream_t s);
hipError_t launch_query(const QueryArgs& a, int n_wg, hipStream_t s);
hipError_t launch_exchange(const ExchangeArgs& a, int n_wg, hipStream_t s);
hipError_t launch_anchor_points(const float* x, int64_t n, int D, const float* x_anc, float* xa, hipStream_t s);
hipError_t launch_master_counts(const SubDev* subs, const int32_t* counts, int n_sub, int32_t* out, hipStream_t s);
hipError_t launch_evaluate(const EvalArgs& a, hipStream_t s);

// Kernel entry points and their LDS needs (for graph nodes and occupancy).
const void* step_kernel_ptr(const Shape& sh, int tile_points);
const void* query_kernel_ptr(const Shape& sh, int what, int small = 0);   // what: Q_VALUE, Q_UVPW, Q_CHANNELS/Q_RESIDUAL
const void* exchange_kernel_ptr(const Shape& sh);
const void* prep_kernel_ptr();
const void* slab_sum_kernel_ptr();
const void* grad_kernel_ptr();
const void* clip_kernel_ptr();
const void* adam_kernel_ptr();
void grid_slab_sum(const ReduceArgs& a, dim3* grid, dim3* block);
int step_lds_floats(const Shape& sh, int tile_points);
int query_lds_floats(const Shape& sh, int small = 0);
int step_value_points(int dim, int tile_points);
void grid_prep(const PrepArgs& a, dim3* grid, dim3* block);
void grid_reduce(const ReduceArgs& a, dim3* grid, dim3* block);

}  // namespace ddp
