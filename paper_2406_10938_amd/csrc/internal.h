// Internal host-side interface between the C ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

// ---- projection (k_project.hip) ----
enum { PROJ_COLMAJOR = 0, PROJ_ROWMAJOR = 1, PROJ_ENCODE = 2 };

struct ProjectArgs {
    const float* X = nullptr;        // M x d (or rows gathered through `rows`)
    const uint16_t* Xbf = nullptr;   // BF16 copy when bf16
    const int32_t* rows = nullptr;
    int64_t M = 0;
    int d = 0;
    const float* A = nullptr;        // N x d
    const uint16_t* Abf = nullptr;
    int N = 0;
    int bf16 = 0;
    float* Pout = nullptr;
    int64_t ldp = 0;
    const float* E = nullptr;        // [N][N_r+1] edge table
    int N_r = 0;
    int K = 0;
    uint8_t* codes = nullptr;        // [L][n][K]
    int64_t n_codes = 0;
};

hipError_t dl_launch_project(const ProjectArgs& a, int mode, hipStream_t st);
hipError_t dl_launch_to_bf16(const float* x, uint16_t* y, int64_t cnt, hipStream_t st);
// xe (optional): squared norm of each row's BF16 rounding error.
hipError_t dl_launch_row_norms(const float* X, int64_t n, int d, float* xn, float* xn_bf, float* xe, uint16_t* xbf,
                               hipStream_t st);
// Bit pattern of the largest of n non-negative floats into *out (which the
// launch clears first).
hipError_t dl_launch_max_f32(const float* v, int64_t n, uint32_t* out, hipStream_t st);

// ---- sorting and scans (k_sort.hip) ----
size_t dl_scan_tmp_bytes(int64_t n);
hipError_t dl_exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, uint32_t* total,
                             hipStream_t st);
size_t dl_radix_tmp_bytes(int64_t n);
hipError_t dl_radix_sort_pairs(uint32_t* keys, uint32_t* vals, int64_t n, int lo_bit, int hi_bit, void* tmp,
                               hipStream_t st);
size_t dl_breakpoint_tmp_bytes(int64_t n_s, int N);
hipError_t dl_breakpoints(const float* Ps, int64_t n_s, int N, int N_r, float* B, float* E, void* tmp,
                          hipStream_t st);
hipError_t dl_edges_from_breakpoints(const float* B, float* E, int N, int N_r, hipStream_t st);

// ---- trees (k_tree.hip) ----
// A tree is built in three phases, so that the L trees of an index can run
// interleaved with one host wait per phase boundary (the next phase's launch
// shape is a count the previous one leaves on the device): runs (totals[0]
// runs), split (totals[1] leaves), leaves (the leaf table).  Each tree keeps
// its own tmp of dl_tree_tmp_bytes(n, K) bytes through all three.
size_t dl_tree_tmp_bytes(int64_t n, int K);
hipError_t dl_tree_runs(const uint8_t* codes_i, int64_t n, int K, int N_r, int32_t* perm, uint8_t* scodes,
                        void* tmp, uint32_t* totals, hipStream_t st);
// phase 2 of the L trees together (L <= 8): nruns[i] from phase 1; the leaf
// count of tree i goes to totals[2 i + 1]
hipError_t dl_tree_split_all(int L, int64_t n, int K, int N_r, int max_leaf, int32_t* const* perm,
                             uint8_t* const* scodes, void* const* tmp, const uint32_t* nruns, uint32_t* totals,
                             hipStream_t st);
hipError_t dl_tree_leaves(int64_t n, int K, int N_r, const uint8_t* scodes, void* tmp, uint32_t nruns, uint32_t nl,
                          int32_t* leaf_start, uint8_t* leaf_lo, uint8_t* leaf_hi, hipStream_t st);

// ---- query (k_query.hip) ----
// Leaf tables of the L DE-Trees: leaf_of[i*n + o] is the leaf of point o in
// tree i; start[i] (leaves+1 offsets into perm + i*n), lo[i]/hi[i] (leaves x K
// region codes of the leaf's prefix box).
struct LeafTabs {
    const int32_t* leaf_of = nullptr;
    const int32_t* perm = nullptr;
    const int32_t* start[8] = {};
    const uint8_t* lo[8] = {};
    const uint8_t* hi[8] = {};
};

// Running minima stored per candidate when S stays implicit: the minimum of
// the per-tree bounds over trees 1..L-2 (when L >= 3) and over trees 1..L-1.
constexpr int dl_prefix_mins(int L) { return L >= 3 ? 2 : 1; }

struct QueryArgs {
    int L = 0, K = 0, N_r = 0, d = 0;
    int64_t n = 0;
    const float* E = nullptr;
    const uint8_t* codes = nullptr;
    const float* X = nullptr;
    const uint16_t* Xbf = nullptr;
    const float* Q = nullptr;        // all queries, nq x d
    const float* Qp = nullptr;       // all projected queries, nq x L*K
    int64_t q0 = 0;                  // first query of the chunk
    int nqc = 0;                     // queries in the chunk
    int G = 0;                       // guess subset size
    const uint8_t* gcodes = nullptr; // codes of the guess subset, [L][G][K]
    const int32_t* gleaf = nullptr;  // leaves of the guess subset, [L][G]
    int leaf = 0;                    // candidates by leaf boxes (leaf granularity)
    LeafTabs lt;
    float* gm = nullptr;             // nqc x G guess values
    uint64_t guess_rank = 0;
    uint64_t N_S = 0;
    int k = 0;
    int64_t cap = 0;                 // candidate slots per query
    int64_t all_n = 0;               // > 0: S = D (every point), skip filter/select
    // workspace (per chunk, indexed by query within the chunk)
    float* gthr = nullptr;
    uint32_t* counts = nullptr;
    int32_t* cand_id = nullptr;
    float* cand_m = nullptr;         // m^2 = min over trees of the bounds
    int32_t* cand_ft = nullptr;      // first admitting tree of each member of S
    uint8_t* cand_f8 = nullptr;      // first admitting tree per candidate where the exact stop pass ran
    float* cand_lb = nullptr;        // L bounds per candidate; with an implicit S dl_prefix_mins(L) running minima
    int32_t* status = nullptr;
    unsigned long long* stat = nullptr;   // profiling counters on the device (null when off): see dl_stat_ptr
    uint32_t* s_count = nullptr;
    float* thr = nullptr;
    int32_t* stop = nullptr;
    uint64_t* ws = nullptr;
    // masked dense verification
    uint64_t* bm = nullptr;          // per query, ceil(n/64) words: bit o = o in S
    int64_t W = 0;
    float* tau = nullptr;            // per query upper bound on the k'-th squared distance
    float* qn = nullptr;             // per query squared norm
    uint16_t* Qbf = nullptr;         // chunk's queries in BF16 (dense_bf16)
    const float* xn = nullptr;       // squared norms of the rows
    const float* xn_bf = nullptr;    // squared norms of the BF16 rows
    int dense_bf16 = 0;
    float margin_c = 0.f;
    // 0: the selection leaves S implicit in the candidate list (members are the
    // entries with 1 <= f(o) <= the stop tree; dense point-granularity path)
    int compact_s = 1;
    // FP32 form screened with BF16 products: tau is widened per query to
    // (sqrt(tau) (1 + tau_rel) + ||q - bf16(q)|| + emax)^2, times slack
    int widen_tau = 0;
    float tau_rel = 0.f;
    float emax = 0.f;                // bound on the largest ||o - bf16(o)||
    uint32_t* svc = nullptr;         // survivors per query
    int32_t* sv = nullptr;
    int64_t cap_sv = 0;
    // printed radius ladder (FIXED r_min)
    int fixed = 0;
    const float* rad2 = nullptr;     // (eps r_min c^t)^2, t < T
    const float* c2 = nullptr;       // (c r_min c^t)^2, t < T
    int T = 0;
    // MFMA screen of the range filter and its exact pass
    const uint16_t* ballb = nullptr;  // point vectors of the screen, FP16 [L][n][KB]
    uint16_t* uqb = nullptr;          // the chunk's query vectors, FP16 [L][nqc][KB]
    const uint8_t* codes_pm = nullptr;   // codes point-major, [n][L*K] (exact pass of the screen)
    // outputs (all queries)
    int64_t* out_ids = nullptr;
    float* out_d = nullptr;
};

bool dl_supported_lk(int L, int K);
// Range filter as an MFMA screen (a ball around each clamped cell) followed by
// the exact bound of the pairs it keeps (k_ball.hip); same output as
// dl_launch_filter for the magic radius at point granularity.
bool dl_ball_supported(int L, int K);
int dl_ball_width(int K);   // KB: FP16 values per vector and tree
// codes [L][n][K] -> point-major [n][L*K]
hipError_t dl_launch_codes_point_major(const uint8_t* codes, int64_t n, int L, int K, uint8_t* out, hipStream_t st);
// point vectors of the screen, FP16 [L][n][KB]
hipError_t dl_launch_ball_table(const uint8_t* codes, int64_t n, int L, int K, const float* E, int N_r,
                                uint16_t* outb, hipStream_t st);
hipError_t dl_launch_ball_query(const QueryArgs& a, hipStream_t st);
// the screen (survivor words into a.bm) and the exact pass over them
hipError_t dl_launch_ball_screen(const QueryArgs& a, hipStream_t st);
hipError_t dl_launch_ball_exact(const QueryArgs& a, hipStream_t st);
// Issue-rate probe of the range filter's bound arithmetic (L = 4, K = 16):
// `lanes` (a multiple of 256) synthetic cells against nq projected queries.
hipError_t dl_launch_valu_probe(const float* qp, int nq, float* out, int64_t lanes, hipStream_t st);
// p[0..n) = v, on the stream
hipError_t dl_launch_fill_f32(float* p, float v, int64_t n, hipStream_t st);
// the FIXED radius ladder (eps r_t)^2, then (c r_t)^2, r_t = r_min c^t, t < rounds
hipError_t dl_launch_ladder(float* out, int rounds, double eps, double r_min, double c, hipStream_t st);
size_t dl_verify_smem(int d, int k);   // LDS bytes of the gathered verification
hipError_t dl_launch_guess(const QueryArgs& a, hipStream_t st);
// leaf_of of one tree: out[perm[p]] = the leaf whose run holds position p.
hipError_t dl_launch_leaf_of(const int32_t* perm, const int32_t* start, int64_t nleaves, int64_t n, int32_t* blk,
                             int32_t* out, hipStream_t st);   // blk: (n + 255) / 256 int32 of scratch
// Leaves of the guess subset: out[i*G + p] = leaf_of[i*n + o_p].
hipError_t dl_launch_pack_sample_leaves(const int32_t* leaf_of, int64_t n, int L, int G, int32_t* out,
                                        hipStream_t st);
// Packs the codes of the guess subset (G = min(n, 16384) points) as [L][G][K].
hipError_t dl_launch_pack_sample(const uint8_t* codes, int64_t n, int L, int K, int G, uint8_t* out,
                                 hipStream_t st);
hipError_t dl_launch_filter(const QueryArgs& a, hipStream_t st);
hipError_t dl_launch_select(const QueryArgs& a, hipStream_t st);
hipError_t dl_launch_verify(const QueryArgs& a, int want, hipStream_t st);
hipError_t dl_launch_tau(const QueryArgs& a, int64_t T, int kprime, hipStream_t st);
hipError_t dl_launch_dense(const QueryArgs& a, hipStream_t st);
hipError_t dl_launch_final(const QueryArgs& a, hipStream_t st);
// Point granularity: keeps only the members of S among the dense pass's
// survivors (the bitmap holds the filter's hits, a superset of S).
hipError_t dl_launch_survivor_members(const QueryArgs& a, hipStream_t st);
hipError_t dl_launch_fixed_finish(const QueryArgs& a, int32_t* rounds, hipStream_t st);

// ---- kernel timing (detlsh_api.cpp) ----
struct DlTimer {
    int id;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    DlTimer(int id_, hipStream_t st_);
    ~DlTimer();
};
// Profiling counters on device `dev` (summed by the kernels while profiling
// is enabled; null otherwise): [0] screen survivors evaluated by the exact
// pass, [1] those that became candidates.
enum { S_EXACT_SURVIVORS = 0, S_EXACT_CANDIDATES, S_COUNT };
unsigned long long* dl_stat_ptr(int dev);
enum {
    T_PROJECT_SAMPLE = 0, T_BREAKPOINTS, T_ENCODE, T_TREE, T_QPROJECT, T_GUESS, T_FILTER, T_SELECT,
    T_VERIFY, T_BF16, T_TAU, T_DENSE, T_FINAL, T_SCREEN, T_EXACT, T_COUNT
};
