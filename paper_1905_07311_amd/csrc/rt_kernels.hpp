// Launchers of the device kernels used by the host drivers (rtucker.cpp).
// Every launcher enqueues on `stream` and returns the hipError_t of the launch.
// Shapes: a row-major tensor is viewed, for mode n, as (L, J, R) with
// L = prod of dims before n, J = dims[n], R = prod of dims after n; the
// mode-n unfolding has J rows and K = L R columns, column c = l R + r.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rtucker.h"

namespace rt {

constexpr int LMAX = 64;     // largest sketch width / rank handled by the dense FP64 kernels

enum class Dt : int { F32 = 0, F64 = 1 };

struct Shape3 { int64_t L, J, R; };

// ---- sketch:  Y = X_(n) Omega[:, col0 : col0 + ell]  (§2.4 Alg. 1 step 1) ------------
// Writes split-K partial sums to `partial` ([nsplit][J][ell], accumulate type),
// then `reduce_partials` folds them in a fixed order into Y (double, J x ell).
// If nrm2_partial != nullptr, the kernel also accumulates sum x^2 (fp64) per
// workgroup into nrm2_partial[workgroup] (every element is read exactly once).
struct SketchPlan {
    int nsplit;            // split-K factor (gridDim.x)
    int nrowtile;          // gridDim.y
    int64_t tiles_per_split;
    size_t partial_elems;  // nsplit * J * ldp
    int nwg;               // nsplit * nrowtile
    int kind;              // kernel variant: 0 generic (LDS-staged VALU), 1 MFMA float32,
                           // 3 float32-accurate from three bfloat16 pieces (16x16x32 MFMA, six products),
                           // 4 the bfloat16 sketch: two bfloat16 pieces, three products, same kernel
    int rb;                // MFMA variant: 64-row blocks per wave (1, 2 or 4); kind 3: 16-row blocks
    int rw;                // MFMA variant: row blocks per workgroup (1 or 2)
    int nq;                // MFMA variant: compiled column quads (ell <= 4 nq); kind 3: 16-column blocks
    int ldp;               // row length of a partial (ell, or 4 nq for the MFMA kernel)
    int kc = 32;           // kinds 3 and 4: unfolding columns per tile (32 or 64)
};
// split3: allow the float32 kernel built on bfloat16 pieces (kind 3; not for explicit Omega)
SketchPlan plan_sketch(Dt dt, int prec, Shape3 s, int ell, int64_t col0, const void* X, bool split3 = true);
hipError_t launch_sketch(const SketchPlan& p, Dt dt, int prec, const void* X, Shape3 s, int ell,
                         int64_t col0, uint64_t seed, uint32_t mode, void* partial,
                         double* nrm2_partial, hipStream_t stream);

// Y = X_(n) Z with Z[l R + r][k] = Om[(l ell + k) R + r] (Om: (L, ell, R), dtype dt),
// split-K partials as launch_sketch.  Plan: plan_sketch with prec 0 (the generic
// kernel) or, for float data with R % 4 == 0 and a 16-byte aligned Om, prec 1
// (the MFMA rows kernel).
hipError_t launch_sketch_explicit(const SketchPlan& p, Dt dt, const void* X, Shape3 s, int ell, const void* Om,
                                  void* partial, hipStream_t stream);

// out[e] = sum_{s < nparts} in[s * n + e] (in float or double, summed in fp64 in
// the order s = 0, 1, ...).  out is double.
// tmp: ceil(nparts / 32) * n doubles of scratch (needed when nparts > 32)
hipError_t launch_reduce_partials(const void* in, bool in_is_f64, int64_t nparts, int64_t n,
                                  double* out, hipStream_t stream, double* tmp);
// The same for parts of `rows` rows of `ldin` elements of which the first `cols`
// are summed: out[i * cols + k] = sum_s in[(s * rows + i) * ldin + k].
hipError_t launch_reduce_rows(const void* in, bool in_is_f64, int64_t nparts, int64_t rows, int64_t cols,
                              int64_t ldin, double* out, hipStream_t stream, double* tmp);
inline size_t reduce_partials_tmp(int64_t nparts, int64_t n) { return nparts > 32 ? (size_t)((nparts + 31) / 32) * n : 0; }
// out[0] = sum of `n` doubles (single workgroup, fixed order of a tree)
hipError_t launch_sum_scalar(const double* in, int64_t n, double* out, hipStream_t stream);

// ---- orthonormalisation:  Q = orth(Y)  (§2.4 Alg. 1 step 2) --------------------------
// In place on Y (double, J x ell, row-major, ld = ell).  CholeskyQR2 over many
// workgroups; a sketch it does not accept goes to one workgroup running
// shifted CholeskyQR3 and then Householder QR, which pads a numerically rank
// deficient Y with zero-weight orthonormal directions.  Optionally writes a
// float copy Qf.  status[0] is
// set to a bit mask: 1 = padded / rank deficient, 2 = fallback path used,
// 4 = non-finite input.
// `accept_ratio`: CholeskyQR2 is accepted when the smallest relative Cholesky pivot of
// the first pass is >= accept_ratio and that of the second pass >= 1/2.
// `scratch`: orth_scratch(J, ell) doubles.
hipError_t launch_orth(double* Y, int64_t J, int ell, float* Qf, double accept_ratio,
                       uint32_t* status, double* scratch, hipStream_t stream);
size_t orth_scratch(int64_t J, int ell);

// ---- projection / core update:  B = G x_n Q^T  (Alg. 1 step 3; Alg. 3 core update) --
// B[l, k, r] = sum_i Q[i, k] G[l, i, r], k < ell; Q is J x ell (row-major, ld = ldq).
// tq: type of Q (F32 or F64); accumulation is in the wider of (X, Q) types.
// If gram_partial != nullptr, each workgroup adds the fp64 Gram sum_c B[:, c] B[:, c]^T
// of its columns to gram_partial[wg][ell][ell]; if nrm2_partial != nullptr, sum B^2
// (fp64) per workgroup.  `nwg_out` receives the workgroup count.
// kind 0 generic, 1 MFMA strips, 2 MFMA rows (R == 1).  The MFMA kinds may split
// the contraction over nsplit workgroup rows (jchunk mode rows each) into float
// partials [nsplit][L][ell][R] (partial_elems floats of workspace) that
// launch_project_reduce adds in a fixed order.
struct ProjectPlan {
    int nwg;
    int64_t ntiles;
    int kind;
    int sets = 1;
    int nsplit = 1;
    int64_t jchunk = 0;
    int64_t split_stride = 0;
    size_t partial_elems = 0;
};
ProjectPlan plan_project(Dt dx, Dt dq, Shape3 s, int ell, const void* G, const void* B, int64_t koff);
// ldj: stride of the mode index in G (= s.J for a plain tensor; larger when only
// the first s.J rows of a wider buffer are contracted).  B is written at
// B[(l * ldk + koff + k) * R + r] (ldk = ell, koff = 0 for a plain tensor).
hipError_t launch_project(const ProjectPlan& p, Dt dx, Dt dq, const void* G, Shape3 s, int64_t ldj,
                          const void* Q, int64_t ldq, int ell, void* B, int64_t ldk, int64_t koff,
                          double* gram_partial, double* nrm2_partial, hipStream_t stream);
// fp64 Gram partials of the first k mode rows of a (L, ldk, R) tensor; nwg from plan_gram3.
int plan_gram3(int64_t L, int64_t R);
hipError_t launch_gram3(const void* B, Dt dt, int64_t L, int64_t ldk, int64_t R, int k, double* partial, int nwg,
                        hipStream_t stream);

// ---- truncation (Alg. 1 steps 4-6) ----------------------------------------------------
// W: ell x ell fp64 Gram of B (from the projection), Q: J x ell fp64.
// Jacobi eigendecomposition of W, eigenvalues sorted in decreasing order.
// Fixed rank: k = r.  Adaptive: k = smallest k with max(E,0) + sum_{t>=k} lambda_t
// <= tau2 (E = *E_dev), capped at kmax.
// Writes U (ell x k, double, and float copy Uf), A = Q U (J x k, in dtype `da`,
// columns sign-fixed: largest-|.| entry positive), lam (ell, sorted eigenvalues),
// kout[0] = k.
// jtol: Jacobi stops when the off-diagonal sum of squares is <= jtol ||W||_F^2.
// kout is required; scratch: truncate_scratch(J, ell) doubles.
hipError_t launch_truncate(const double* W, int ell, const double* Q, int64_t ldq, int64_t J, int r_fixed,
                           const double* E_dev, double tau2, double* U, float* Uf, void* A, Dt da,
                           double* lam, int* kout, double jtol, double* scratch, hipStream_t stream);
size_t truncate_scratch(int64_t J, int ell);

// ---- subspace iteration: orthonormal rows of B via the eigendecomposition of W = B B^T --
// W (ell x ell fp64, symmetric PSD) = V diag(lam) V^T; T[i][k] = V[i][k] /
// sqrt(max(lam_k, drop lam_max)) (T and the float copy Tf, row-major ell x ell; zero
// when W = 0), so that T^T B has orthonormal rows along the directions above the floor.
// jtol as launch_truncate.
hipError_t launch_svqb(const double* W, int ell, double drop, double* T, float* Tf, double jtol, hipStream_t stream);

// ---- structure-preserving STHOSVD (Alg. 6): row selection on Q -------------------------
// Q: J x ell fp64 with orthonormal columns.  sel (ell ints, device): the pivoted-QR
// rows of Q then strong-RRQR exchanges until every |A| <= eta, A = Q Q[sel]^-1 written
// to Aout (J x ell, dtype da); swaps[0] = exchanges made.  scratch: 2 J ell doubles.
hipError_t launch_select_rows(const double* Q, int64_t J, int ell, double eta, int max_swaps, double* scratch,
                              void* Aout, Dt da, int* sel, int* swaps, hipStream_t stream);
// The same selection for 512 < J <= select_grid_rows(): one cooperative grid of
// ceil(J / 256) workgroups with a grid-wide barrier per step (identical result).
int64_t select_grid_rows();
hipError_t launch_select_rows_grid(const double* Q, int64_t J, int ell, double eta, int max_swaps, double* scratch,
                                   void* Aout, Dt da, int* sel, int* swaps, hipStream_t stream);
// out (L, ell, R) = G (L, J, R) at the mode indices sel[0..ell) (dtype dt)
hipError_t launch_gather_mode(const void* G, Dt dt, Shape3 s, const int* sel, int ell, void* out, hipStream_t stream);

// ---- sparse (COO) steps of SP-STHOSVD (Alg. 6, §5) ------------------------------------
// Entry e of a COO tensor: coordinates idx[m * ldi + e] (int32), value vals[e].
// nnz_dev: the entry count on the device (NULL: `bound` itself); bound: an upper
// bound used to size grids.  Entries with a coordinate outside dims are skipped.
struct CooDims { int32_t d; int64_t dims[RT_MAXD]; };
int64_t coo_chunks(int64_t bound);   // compaction chunks (length of cnt / off)
// status |= bit when some entry has a coordinate out of range
hipError_t launch_coo_check(const int32_t* idx, int64_t ldi, int64_t nnz, const CooDims& cd, uint32_t* status,
                            uint32_t bit, hipStream_t stream);
// Y (J x ell, double, zeroed by the caller) += G_(mode) Omega[:, col0 : col0 + ell]
hipError_t launch_coo_sketch(const int32_t* idx, int64_t ldi, const void* vals, Dt dt, const int64_t* nnz_dev,
                             int64_t bound, const CooDims& cd, int mode, int ell, int64_t col0, uint64_t seed,
                             double* Y, hipStream_t stream);
// The same sketch for an input core of nnz entries (count on the host), the
// entries first grouped by blocks of 2^shift rows (so each block's rows are
// accumulated in LDS and added to Y once).  Scratch: hist (nch x nbk int32), off
// (nch x nbk int64), bstart and pstart (nbk + 1 int64 each), keys and rv (nnz
// int64 / double).  ok: the plan fits (J and ell small enough for LDS blocks).
struct BinPlan { int shift; int nbk; int64_t nch; bool ok; };
BinPlan plan_coo_bins(int64_t J, int ell, int64_t nnz);
hipError_t launch_coo_sketch_binned(const BinPlan& bp, const int32_t* idx, const void* vals, Dt dt, int64_t nnz,
                                    const CooDims& cd, int mode, int ell, int64_t col0, uint64_t seed, double* Y,
                                    int32_t* hist, int64_t* off, int64_t* bstart, int64_t* pstart, int64_t* keys,
                                    double* rv, hipStream_t stream);
// G_(mode) <- P^T G_(mode): the entries whose mode coordinate is sel[j] for some j,
// in input order, with that coordinate replaced by j, into (idx_out, ldo,
// vals_out); their count into *nnz_out.  inv: dims[mode] ints; cnt, off:
// coo_chunks(bound) int64 each (scratch).
hipError_t launch_coo_restrict(const int32_t* idx, int64_t ldi, const void* vals, Dt dt, const int64_t* nnz_dev,
                               int64_t bound, const CooDims& cd, int mode, const int* sel, int ell, int32_t* inv,
                               int64_t* cnt, int64_t* off, int32_t* idx_out, int64_t ldo, void* vals_out,
                               int64_t* nnz_out, hipStream_t stream);
// out (dense row-major dims, zeroed by the caller) += the entries
hipError_t launch_coo_densify(const int32_t* idx, int64_t ldi, const void* vals, Dt dt, const int64_t* nnz_dev,
                              int64_t bound, const CooDims& cd, void* out, hipStream_t stream);

// ---- adaptive block step (reading of AdaptRangeFinder, §4) ----------------------------
// Y (J x b, double) is orthogonalised twice against Qall[:, :k] (J x ld, double),
// then orthonormalised with a rank-revealing drop (singular values <= drop * ||Y_in||_F
// are dropped).  The kept columns are appended to Qall at column k and columns
// k + kept .. k + b - 1 are zeroed; knew[0] = kept; Qf (optional, J x ld floats)
// gets the float copy of these b columns.
// `scratch`: 2 J b doubles.  y0_ext (device, optional): the norm the drop rule
// compares with, when Y was already projected against earlier basis columns.
hipError_t launch_block_orth(double* Y, int64_t J, int b, double* Qall, int ldq, int k,
                             double drop, int* knew, float* Qf, double* scratch, hipStream_t stream,
                             const double* y0_ext = nullptr);
// one-time per-device set-up of the single-workgroup dense kernels (LDS > 64 KiB)
hipError_t dense_init();

// ---- MFMA variants (float32 data, v_mfma_f32_4x4x1_16b) -------------------------------
bool sketch_mfma_ok(Shape3 s, int ell, int64_t col0, const void* X);
hipError_t launch_sketch_f32_rows(const SketchPlan& p, const float* X, Shape3 s, int ell, int64_t col0,
                                  uint64_t seed, uint32_t mode, float* partial, double* nrm2, hipStream_t stream);
hipError_t launch_sketch_f32_cols(const SketchPlan& p, const float* X, Shape3 s, int ell, int64_t col0,
                                  uint64_t seed, uint32_t mode, float* partial, double* nrm2, hipStream_t stream);
// kind 3: each float32 operand split into three bfloat16 pieces, six piece
// products per product on v_mfma_f32_16x16x32_bf16 (float32 accuracy); needs
// J > 64, 1 <= ell <= 64, col0 % 4 == 0, R % 8 == 0, 16-byte aligned X of at most
// 0x7fff0000 bytes.  Partials have ldp = ell.  bf16 (kind 4): the bfloat16
// sketch, two truncated bfloat16 pieces per operand and the three products of
// weight above 2^-16 (hh, hm, mh), relative accuracy about 2^-15.
bool sketch_x6_ok(Shape3 s, int ell, int64_t col0, const void* X);
// rb (16-row blocks per wave: 1, 2 or 4) and wgs (workgroups the column split
// aims for): 0 = the built-in rule
void plan_sketch_x6(SketchPlan& p, Shape3 s, int ell, bool bf16, int rb = 0, int wgs = 0);
// Process-wide tile table (rt_tuning_set / rt_tuning_plan).
rt_status tuning_set(const rt_tune_entry* entries, int32_t n);
// plan_sketch's choice for a shape, and whether a table entry made it
SketchPlan plan_sketch_info(Dt dt, int prec, Shape3 s, int ell, int64_t col0, const void* X, bool split3,
                            bool* from_table);
int stride_class(Shape3 s);
hipError_t launch_sketch_f32_x6(const SketchPlan& p, const float* X, Shape3 s, int ell, int64_t col0, uint64_t seed,
                                uint32_t mode, float* partial, double* nrm2, hipStream_t stream);
// explicit Omega from Om ((L, ell, R) float tensor, 16-byte aligned); needs R % 4 == 0
hipError_t launch_sketch_f32_rows_explicit(const SketchPlan& p, const float* X, Shape3 s, int ell, const float* Om,
                                           float* partial, hipStream_t stream);
bool project_mfma_ok(Shape3 s, int ell, const void* G, const void* B, int64_t koff);
void plan_project_mfma(ProjectPlan& p, Shape3 s, int ell);
// with p.nsplit > 1, B is the partial buffer (ldk = ell, koff = 0) and nrm2 must be null
hipError_t launch_project_mfma(const ProjectPlan& p, const float* G, Shape3 s, int64_t ldj, const float* Q, int64_t ldq,
                               int ell, float* B, int64_t ldk, int64_t koff, double* nrm2, hipStream_t stream);
// last mode (R == 1): B (L x ldk, columns koff..) = G (L x J, row stride ldj) Q
void plan_project_r1_mfma(ProjectPlan& p, Shape3 s, int ell);
hipError_t launch_project_r1_mfma(const ProjectPlan& p, const float* G, Shape3 s, int64_t ldj, const float* Q,
                                  int64_t ldq, int ell, float* B, int64_t ldk, int64_t koff, double* nrm2,
                                  hipStream_t stream);
// B (L, ldk, R) at koff = sum of the nsplit float partials; nrm2 partials per workgroup (nwg)
int plan_project_reduce(int64_t n);
hipError_t launch_project_reduce(const float* part, int nsplit, Shape3 s, int ell, float* B, int64_t ldk, int64_t koff,
                                 double* nrm2, int nwg, hipStream_t stream);

// ---- misc ------------------------------------------------------------------------------
// sum x^2 (fp64) of n elements, per workgroup partials (nwg <= 1024)
int plan_norm(int64_t n);
// Scalars read back at the end of a decomposition (one pinned, device-mapped block).
struct FinishScalars { double nx2, ng2; uint32_t status[RT_MAXD]; };
// End of a decomposition in one workgroup: copies the core (n elements) from
// `core` to `out` when copy is set, sums its squares in fp64 (over the npart
// per-workgroup partials of launch_norm2 when `partial` is given, else over the
// elements, in a fixed order) and writes {*nx2, that sum, status[0 .. RT_MAXD)}
// into `hs`, a pinned host block mapped for the device; visible to the host
// once the stream has been synchronised.  Serves cores of up to
// FINISH_DIRECT_MAX elements directly (larger ones: copy and launch_norm2 first).
constexpr int64_t FINISH_DIRECT_MAX = 1 << 16;
hipError_t launch_finish(const void* core, void* out, Dt dt, int64_t n, bool copy, const double* partial, int npart,
                         const double* nx2, const uint32_t* status, FinishScalars* hs, hipStream_t stream);
hipError_t launch_norm2(const void* X, Dt dt, int64_t n, double* partial, int nwg, hipStream_t stream);
// Mode expansion of reconstruction: out (L, I, R) with out[l, i, q] =
// sum_k A[i, k] G[l, k, q] for G viewed as (L, s.J = r, R) and A (I x r,
// row-major); every R, within the grid limits of expand_ok.
bool expand_ok(Shape3 s, int64_t I);
hipError_t launch_expand(Dt dt, const void* G, Shape3 s, const void* A, int64_t I, void* out, hipStream_t stream);
// AT (cols x rows) = A^T for a row-major rows x cols matrix A, in dtype dt
hipError_t launch_transpose(const void* A, int64_t rows, int64_t cols, void* AT, Dt dt, hipStream_t stream);

// Fixed-rank steps for RT_LMAX < ell <= RT_LMAX_FIXED (rt_wide.hip).
hipError_t launch_wide_copy_cols(const double* src, int64_t J, int w, double* dst, int ldd, int off,
                                 hipStream_t stream);
size_t wide_orth_scratch(int64_t J, int n);
hipError_t launch_wide_orth(double* Y, int64_t J, int n, float* Qf, double accept_ratio, uint32_t* status,
                            double* scratch, hipStream_t stream);
int plan_wide_gram(int64_t K);
hipError_t launch_wide_gram(const void* B, Dt dt, int64_t L, int n, int64_t ldb, int64_t R, double* part, int nwg,
                            hipStream_t stream);
hipError_t launch_wide_eig(const double* W, int n, double tol, double* U, double* lam, hipStream_t stream);
hipError_t launch_wide_factor(const double* Q, int64_t ldq, int64_t J, int n, const double* U, int r, double* A64,
                              double* sgn, void* Aout, Dt da, double* Us, float* Usf, hipStream_t stream);
hipError_t launch_wide_cgs(double* Y, int64_t J, int b, const double* Q, int ldq, int ka, double* y0,
                           hipStream_t stream);
// dst (dtype) <- src (double), n elements
hipError_t launch_cast_from_f64(const double* src, void* dst, Dt dt, int64_t n, hipStream_t stream);
// explicit Omega (testing): out[i][j] = Omega[c0 + i, col0 + j], fp32 or fp64 transform
hipError_t launch_omega(uint64_t seed, uint32_t mode, int64_t c0, int64_t nrows, int64_t col0, int ncols,
                        void* out, Dt dt, hipStream_t stream);
// raw Philox words (testing): out[4 i + t] = word t of block (c0 + i, q, mode)
hipError_t launch_philox_words(uint64_t seed, uint32_t mode, int64_t c0, int64_t n, uint32_t q,
                               uint32_t* out, hipStream_t stream);
// Tucker reconstruction helper is the projection kernel with the factor in place of Q^T.

// ---- grouped execution: one launch serves the same step of many requests ----------------
// Used by the serving executor.  Every launch has a fixed grid (so one
// captured graph serves every iteration) and takes its work from descriptor
// arrays in device memory, refreshed by one host-to-device copy per iteration;
// a request's work is split by its own shape only, so its result does not
// depend on the other requests of the group.  Scalars the host needs come back
// through a mapped pinned slot per request (GRead).
struct GRead {
    int knew;              // kept columns of the block step
    int kfinal;            // rank chosen by the truncation
    double bnorm2;         // ||B_i||^2 of the block's projection (fp64)
    double xnorm2;         // ||G||^2 summed by the first block's sketch
    double gnorm2;         // ||G'||^2 of the truncated core
};
// Adaptive block step: Y = G_(n) Omega[:, col0 : col0 + b] (LDS-staged sketch,
// split-K partials), its fixed-order sum (with ||G||^2 when nrm_partial is set),
// the block orthonormalisation against Qall[:, :kcols] and the projection of G
// on the new columns (a GProj entry).
struct GBlock {
    const float* G;
    int64_t L, J, R;
    int64_t col0;
    uint64_t seed;
    uint32_t mode;
    int b;
    int nsplit, nrowtile;
    int64_t tiles_per_split;
    int64_t wi0;            // first sketch work item (prefix over the group)
    float* partial;         // nsplit * J * b
    double* nrm_partial;    // nsplit * nrowtile, or null
    double* Y;              // J x b
    double* Qall;           // J x cap (fp64)
    float* Qallf;           // J x cap (float copy)
    int cap, kcols;
    double drop;
    int* knew;              // device copy of the kept count
    GRead* rb;
};
// B (L, ldo, R) rows koff .. koff + ell = Q^T G over the first J mode rows of G
// (L, ldj, R), Q float (J x ell, ld ldq); ell from *ell_dev when set (a rank
// chosen on the device; at most ellmax).  Work items: column tiles of 256 x
// chunks of 8 output rows; nrm_partial[item] = fp64 sum of squares of the item's
// outputs, summed into *rb_norm (mapped) by the sum launch.
struct GProj {
    const float* G;
    int64_t L, J, R, ldj;
    const float* Q;
    int64_t ldq;
    int ellmax;
    const int* ell_dev;
    float* out;
    int64_t ldo, koff;
    int64_t wi0;
    int nct, nch;
    double* nrm_partial;
    double* rb_norm;
};
// Truncation of a mode: fp64 Gram of B rows 0 .. kcols (column chunks into
// partials), its eigendecomposition, the rank (smallest k with max(E, 0) + tail
// <= tau2), A = Qall U_k with the sign fix (float, J x k), U_k (float, kcols x k).
struct GTrunc {
    const float* B;
    int64_t L, ldk, R;
    int kcols;
    const double* Qall;
    int64_t J;
    int cap;
    double E, tau2;
    int64_t wi0;            // first Gram work item
    int nchunk;             // Gram column chunks
    double* gpart;          // nchunk * kcols * kcols
    float* A;               // J x k
    float* Uf;              // kcols x k, row stride kcols
    int* kout;
    GRead* rb;
};
struct GHeader {
    int nblock, ntrunc, nbproj, ncproj;
    int64_t sketch_items, bproj_items, gram_items, cproj_items;
};
// Layout of the descriptor buffer: GHeader, then maxreq GBlock, maxreq GProj
// (block projections), maxreq GTrunc, maxreq GProj (core projections).
size_t group_desc_bytes(int maxreq);
// The launches of one iteration (fixed grids; empty lists return at once).
hipError_t launch_group_iteration(const void* desc_dev, int maxreq, int block, hipStream_t stream);
// Sketch plan of one block (generic kernel): nsplit, nrowtile, tiles_per_split.
void group_sketch_plan(int64_t L, int64_t J, int64_t R, int b, int& nsplit, int& nrowtile, int64_t& tps);
// Largest J the grouped block step serves for block width b.
int64_t group_block_maxj(int b);
// Gram column chunks of a truncation over K columns.
int group_gram_chunks(int64_t K);
// the launches of the iteration, by file
hipError_t launch_group_sketch(const GHeader* hdr, const GBlock* d, int block, hipStream_t stream);
hipError_t launch_group_dense(const GHeader* hdr, const GBlock* blk, const GTrunc* tr, int maxreq, hipStream_t stream,
                              int stage);
hipError_t launch_group_tensor(const GHeader* hdr, const GBlock* blk, const GProj* bproj, const GTrunc* tr,
                               const GProj* cproj, int maxreq, hipStream_t stream, int stage);

// ---- allocation-free entry point ---------------------------------------------------------
// Device address of the library's static scratch array on `device` (the current
// device), taken once per device; rt_create calls it.
hipError_t noalloc_init(int device);
// Context accessors and the sketch's argument checks, shared by the entry points.
hipStream_t ctx_stream(const rt_ctx* c);
int ctx_device(const rt_ctx* c);
rt_status check_sketch_args(const rt_ctx* ctx, const rt_tensor* X, int32_t mode, int32_t ell, int64_t col0,
                            rt_precision prec, const double* Y);
rt_status set_error(rt_status s, const char* msg);

}  // namespace rt
