// The library context behind the opaque gspm_ctx handle.
#pragma once

#include <string>
#include <vector>

#include "common.h"
#include "mpnn.h"

namespace gspm {

// Which solve a CG call belongs to, for the iteration-count predictor that
// sizes the first batch of iterations launched before polling.
enum SolveKind { SK_MECH = 0, SK_GS1 = 1, SK_GS2 = 2, SK_GS3 = 3, SK_OTHER = 4, SK_MS = 5, SK_COUNT = 6 };

// offsets (in n) of the GS stages' corrections in DeviceBuffers::gcorr: three,
// two and three components
constexpr int kGcorrOff[3] = {0, 3, 5};

struct DeviceBuffers {
    double *x = nullptr;          // 3n coordinates
    ushort4 *lconn = nullptr;
    int32_t *blk_ptr = nullptr, *blk_nmag = nullptr, *halo_ptr = nullptr, *halo_ids = nullptr, *halo_lo = nullptr;
    uint8_t *img = nullptr;
    double *w = nullptr;
    double *stc64 = nullptr;
    float *stc32 = nullptr;
    uint4 *seg_ent = nullptr;
    uint32_t *seg_off = nullptr;
    uint16_t *seg_nel = nullptr;
    int32_t *seg_ptr = nullptr, *seg_nmag = nullptr;
    double *m = nullptr, *mnext = nullptr, *u = nullptr, *unext = nullptr;   // 3n each
    double *ms = nullptr, *g = nullptr, *gs = nullptr, *b = nullptr, *ch2 = nullptr;
    double *r = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr;
    double *sums = nullptr;       // 9 x kShards
    double *esums = nullptr;      // 4 x kShards
    double *dm = nullptr;         // kShards
    Derived *der = nullptr;       // [2]: stage at m^n, stage at m*
    int32_t *bad = nullptr;
    double *cg_rr = nullptr, *cg_pq = nullptr, *cg_bb = nullptr, *cg_rq = nullptr, *cg_qq = nullptr;
    int32_t *cg_flags = nullptr;  // done[3], iters[3]
    // mixed form: FP32 inner-solve vectors and scalars
    float *r32 = nullptr, *p32 = nullptr, *p32b = nullptr, *q32 = nullptr, *x32 = nullptr;
    double *cgi_rr = nullptr, *cgi_pq = nullptr, *cgi_bb = nullptr, *cgi_rq = nullptr, *cgi_qq = nullptr;
    double *r2 = nullptr, *q2 = nullptr;          // 3n: second r and q of the single-reduction elastic CG
    float *r32b = nullptr, *q32b = nullptr;       // 3n: the same for the FP32 inner solves
    int32_t *cgi_flags = nullptr;
    double *mprev = nullptr;      // 3n: m^{n-1} (previous committed state), for the learned warm start
    double *uprev = nullptr;      // 3n: u^{n-2}, for the previous displacement increment
    double *gcorr = nullptr;      // 8n: the last step's GS corrections (solution - lumped start): stages 1, 2, 3
                                  // at kGcorrOff[stage] * n
    double *gstart = nullptr;     // 3n: the start of the running GS solve
    double *du_prev = nullptr;    // 3n: u^{n-1} - u^{n-2} (warm start scratch)
    double *kdu = nullptr;        // 3n: K (u^{n-1} - u^{n-2}) (warm start scratch)
    double *wred = nullptr;       // kMrSums x kShards: minimum-residual sums
    double *wcoef = nullptr;      // 2: coefficients of the last minimum-residual start
    double *ud = nullptr, *udnext = nullptr;   // n: local magnetostatic potential (committed, in progress)
    int32_t *rep = nullptr;       // n: the first caller node of each unique node
    double *cg_rz = nullptr, *cgi_rz = nullptr;   // r . D^-1 r rings of the Jacobi-preconditioned GS solves
    double *cg_rzq = nullptr, *cg_qzq = nullptr, *cgi_rzq = nullptr, *cgi_qzq = nullptr;   // r.D^-1 q, q.D^-1 q rings
    // deterministic mode: the fixed-order sums' slots and per owned node its element copies (MeshView)
    double *det_part = nullptr;
    double **det_dst = nullptr;
    int32_t *det_count = nullptr;
    int32_t *inc_ptr = nullptr;
    uint16_t *inc_ent = nullptr;
    // the GS operator in row form (GsRowsHost): the pattern, K and M (FP64),
    // and per slot the combined coefficients of one (eps, mass) pair in FP64
    // and (mixed contexts) FP32
    int32_t *gs_off = nullptr;
    uint16_t *gs_col = nullptr;
    int32_t *gs_halo_ptr = nullptr, *gs_halo_ids = nullptr;   // the row blocks' halo lists
    double *gs_kv = nullptr, *gs_mv = nullptr, *gs_kd = nullptr, *gs_md = nullptr;
    double *gs_a64[2] = {nullptr, nullptr}, *gs_d64[2] = {nullptr, nullptr};
    float *gs_a32[2] = {nullptr, nullptr}, *gs_d32[2] = {nullptr, nullptr};
};

// Which (eps, mass) pair a coefficient slot of the GS rows holds.
struct GsSlot {
    bool valid = false;
    double eps = 0.0, mass = 0.0;
    int64_t used = 0;             // tick of the last use (the least recent slot is rebuilt)
};

// Device state of the learned warm start (allocated on first use).
struct MpnnState {
    bool ready = false, have_params = false;
    int32_t *gptr = nullptr, *gnbr = nullptr;
    int64_t nedges = 0;
    float *master = nullptr, *wr = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;
    uint16_t *mats = nullptr, *acts = nullptr;
    float *y = nullptr;
    double *red = nullptr, *dvec = nullptr, *du = nullptr, *mp_in = nullptr, *m_in = nullptr;
    float *gh = nullptr, *gha = nullptr, *gab = nullptr, *gy = nullptr, *part = nullptr;
    int part_wgs = 0;
    int64_t adam_t = 0;
    mpnn::Graph graph{};
    mpnn::Net net{};
    mpnn::Acts A{};
    mpnn::Grads G{};
};

// The elastic preconditioner's device data and FFT plans (elastic_precond;
// built by set_params: the grid and restriction lists once per mesh, the
// symbol and diagonal whenever the stiffness changes).
struct GreenState {
    bool mesh_ready = false, sym_ready = false;
    double sym_key[37] = {};      // the Voigt stiffness (36) and scale the symbol and diagonal were built for
    GreenView gv{};
    int32_t *rptr = nullptr, *rgrid = nullptr, *rnode = nullptr;
    void *rw = nullptr, *dinv = nullptr, *ainv = nullptr, *grid = nullptr, *spec = nullptr, *work = nullptr;
    double *aux = nullptr;        // 3 x kShards: mean sums; then 3: the pinned node's shift
    size_t work_bytes = 0;
    void *fwd = nullptr, *inv = nullptr, *info = nullptr;   // rocfft_plan, rocfft_plan, rocfft_execution_info
};

}  // namespace gspm

struct gspm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int precision = GSPM_FP64;
    int block_nodes = 0;
    int reorder = GSPM_REORDER_MORTON;
    bool deterministic = false;           // fixed-order sums (gspm_create_opts.deterministic)
    bool profile = false;
    void *(*alloc_fn)(size_t, void *) = nullptr;   // optional device allocator of the caller
    void (*free_fn)(void *, void *) = nullptr;
    void *alloc_user = nullptr;
    std::string err;

    bool have_mesh = false, have_params = false, have_m = false;
    int64_t n0 = 0, ne = 0, ncopies = 0;
    int32_t n = 0, nblk = 0, nmag = 0, p0 = -1;
    double vc = 0.0;
    double box_lo[3] = {0.0, 0.0, 0.0};   // the periodic box's min corner
    std::vector<int32_t> user2int;
    std::vector<double> w_host;   // lumped weights (internal order)

    gspm::DeviceBuffers d;
    char *arena = nullptr;                // one allocation holding the mesh upload's buffers
    size_t arena_size = 0, arena_used = 0;
    bool arena_planning = false;
    gspm::MeshView mv{};
    gspm::MeshView mv_rows{};     // mv with the GS row blocks (size, count, halo lists, largest staging)
    gspm::CGScalars cg{};
    gspm::CGScalars cg_in{};      // inner FP32 solves of the mixed form
    int32_t *h_flags = nullptr;   // pinned host mirror: 2 slots x (done[3], iters[3])
    double *h_mixed = nullptr;    // pinned staging of the mixed form's outer loop
    int64_t refinements = 0;      // outer FP64 residual evaluations that launched an inner solve
    int64_t mech_refinements = 0; // the part of them in elastic solves
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipEvent_t phase_ev[9] = {};          // profile mode: boundaries of a step's phases
    double *h_step = nullptr;             // pinned: the step's results the host reads (sums, flags, residual totals)
    bool want_res = false;                // record the final residual of each solve (the call's last step)
    double last_res[gspm::SK_COUNT] = {}; // relative residual at which the last solve of each kind stopped
    // profile mode: event pairs around the launches of list 0 (the elastic CG
    // iteration, plain or preconditioned matvec) and list 1 (the GS matvec on
    // three components); prof_list names the list the running solve records into
    struct ProfList {
        std::vector<hipEvent_t> ev;
        std::vector<int> iter;    // CG iteration of each timed pair, -1 = dropped
        size_t used = 0;
    } prof[2];
    int prof_list = -1;

    gspm_params p{};
    gspm::Material mat{};
    gspm::DeriveArgs dargs{};
    // iteration counts of the last solve of each kind (first inner solve of a
    // mixed-form solve, or any later one), which size the first batch
    int predict[gspm::SK_COUNT][2] = {{32, 8}, {8, 4}, {8, 4}, {8, 4}, {16, 8}, {32, 8}};
    int refine_slot = 0;                  // 1 while a mixed-form solve runs its second or later inner solve
    bool heavy_iter = false;              // the running solve's iterations are costly (preconditioned): short batches
    int batch_last = -1;                  // the last iteration of the batch being enqueued
    bool pc_owed = false;                 // the preconditioned solve's next batch starts by forming z = B r

    // learned warm start
    gspm::MpnnState nn;
    int warm_mode = GSPM_WARM_PREVIOUS;
    int gs_start = GSPM_GS_START_LUMPED;
    unsigned gcorr_ok = 0;                // bit s: d.gcorr holds GS stage s's last correction
    bool have_prev = false;               // d.mprev holds the state before the last committed step
    int commits = 0;                      // steps committed since the last set_field (u^{n-2} valid from 2)
    std::vector<int32_t> tets_int;        // 4 x ne internal node ids (graph construction)

    double *na_scratch = nullptr;         // this device's scratch of gspm_averages_noalloc (not owned)

    int64_t gs_nent = 0;                  // entries of the GS rows (padding included)
    gspm::GsSlot gs_slot[2];
    int64_t gs_tick = 0;

    gspm::GreenState pc;                  // elastic preconditioner

    ~gspm_ctx();
    void release_mesh();
    void release_nn();
    void release_pc();
};

namespace gspm {

// CG on a prepared right-hand side; see solver.cpp.
struct CgResult {
    int status = GSPM_OK;
    int iters[kMaxComp] = {0, 0, 0};
};

void cg_prepare(gspm_ctx *c, int ns);
CgResult cg_elastic(gspm_ctx *c, double *x, const double *b, double tol, int maxit, SolveKind kind);
CgResult cg_gs(gspm_ctx *c, int nc, double eps, double *x, const double *b, double tol, int maxit, SolveKind kind);
// K^ms x = b (Eq. weak_demag) on nc components, pinned node p0.
CgResult cg_ms(gspm_ctx *c, int nc, double *x, const double *b, double tol, int maxit, SolveKind kind);
int run_steps(gspm_ctx *c, double dt, int nsteps, gspm_step_stats *st);
// The elastic preconditioner: (re)build what the current mesh and parameters
// need (green.cpp); y = B x on FP64 device vectors [3][n] (FP64 contexts).
int green_setup(gspm_ctx *c);
// The GS operator eps K + mass M in row form, its coefficients in FP32
// (mixed contexts only) or FP64; builds the slot on the context's stream when
// the pair is not cached.
GsRowsView gs_rows(gspm_ctx *c, double eps, double mass, bool fp32);
int green_apply64(gspm_ctx *c, const double *x, double *y);
// FFTs of the preconditioner on the context's stream, the two packed complex
// grids as one batch: grid -> spec (forward) or spec -> grid (inverse).
int green_fft(gspm_ctx *c, bool forward);
int hip_check(gspm_ctx *c, hipError_t e, const char *what);
// Device memory of the context: the caller's allocator when given, else hipMalloc / hipFree.
int ctx_malloc(gspm_ctx *c, void **p, size_t bytes, const char *what);
void ctx_free(const gspm_ctx *c, void *p);
// Warm start of the elastic solve on the right-hand side b: x (holding u^{n-1})
// becomes u^{n-1} + a d + c e, d the network's increment at (m, mprev) (when
// mprev != nullptr), e = u^{n-1} - uprev (when uprev != nullptr), (a, c) the
// coefficients minimising |b - K x| (stored at d.wcoef).  Leaves the CG scalars as
// cg_prepare set them.
int minres_start(gspm_ctx *c, const double *m, const double *mprev, const double *uprev, double *x, const double *b);
// Caller-order n0 x 3 <-> internal component-major 3 x n (api.cpp).
int gather_user(gspm_ctx *c, const double *v, std::vector<double> &out);
void scatter_user(const gspm_ctx *c, const std::vector<double> &in, double *out);

}  // namespace gspm
