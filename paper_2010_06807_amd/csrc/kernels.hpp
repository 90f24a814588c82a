// Descriptors shared by the host driver and the HIP kernels, and the launch
// entry points.  All matrices handed to kernels are dense and row-major unless
// a field says column-major.  Pointers are absolute device addresses.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spaqr {

// One rectangular copy: dst[r*ldd + c] = src[r*lds + c] (a plain launch), or
// the transpose dst[c*ldd + r] = src[r*lds + c] (a transposing launch);
// src == nullptr zero-fills (plain launches only).  The tiles of one launch
// must have disjoint destinations: they run concurrently.
template <typename T>
struct CopyTile {
  const T* src;
  T* dst;
  int32_t rows, cols, lds, ldd;
};

// Blocked Householder QR of a row-major m x nc matrix (row stride ld, or nc
// when ld == 0): reflectors for the first n columns, applied to all nc
// columns.  V (unit diagonal implicit) is left below the diagonal and R on and
// above it; tau[0..n) and the compact-WY factors of every JB-column panel
// (JB x JB, column-major, zero-padded) are written.  If some |R_ii| is exactly
// zero, *flag = 1.
template <typename T>
struct QRDesc {
  T* a;
  T* tau;
  T* tpan;
  int* flag;  // may be null
  int32_t m, n, nc, ld;
};

// Trailing update of one column slice of a front whose pivot block was
// factored with nc = n: columns [c0, c0 + cw) of the row-major m-row matrix
// c (row stride ldc) get H_{n-1}^T ... H_0^T, panel by panel from the
// reflectors below the diagonal of the factored pivot block a (row-major, row
// stride ld, a multiple of 16) and the panels' T factors.  For a front c is a
// itself; for the scaling step c is a block to the right of an interface.
// flag (may be null): nonzero skips the item.
template <typename T>
struct TrailDesc {
  const T* a;
  const T* tpan;
  T* c;
  const int* flag;
  int32_t m, n, ld, c0, cw, ldc;
};

// Blocked WY form of 64 reflectors j0 .. j0 + 63 of a factored pivot block a
// (row-major, row stride ld, m rows, n reflectors: V below the diagonal, tau
// their scalars): T_b (64 x 64 row-major) is written to tblk.
template <typename T>
struct WYBlock {
  const T* a;
  const T* tau;
  T* tblk;
  int32_t m, n, ld, j0;
};

// One tile of at most 64 trailing columns [c0, c0 + cw) of the row-major
// m-row matrix c (row stride ldc) to be updated with all n reflectors of the
// factored pivot block a (row stride ld), whose blocks' T_b lie back to back
// at tblk (64 x 64 each).  flag (may be null): nonzero skips the tile.
template <typename T>
struct WYTile {
  const T* a;
  const T* tblk;
  T* c;
  const int* flag;
  int32_t m, n, ld, c0, cw, ldc;
};

// One block B (row-major rows x cols, ld = cols) of the trailing matrix to be
// scaled: B <- U_i^T B (if the row cluster is a scaled interface), then
// B <- B R_j^{-1} (if the column cluster is), or B := I for a scaled
// diagonal block.  Interface factors are column-major P x P with V below the
// diagonal and R_pp on/above it.
template <typename T>
struct ScaleFac {
  const T* vr;
  const T* tau;
  const T* tpan;
  const int* flag;  // nonzero: R_pp had a zero diagonal, interface not scaled
  int32_t P, pad;
  const T* vw;      // the same V row-major (row stride ldw, a multiple of 16), during the stage
  int32_t ldw, pad2;
};

template <typename T>
struct ScaleBlk {
  T* B;             // the block (row-major, ld = cols)
  int32_t rows, cols;
  int32_t fi, fj;   // index into the ScaleFac table, or -1
};

// Zero fill of words 32-bit words at p; block0 = first workgroup of this
// descriptor in a launch over several descriptors.
struct ZeroDesc {
  uint32_t* p;
  int64_t words;
  int64_t block0;
};

// Sparsification of one interface p (Sections 2.5-2.6): gathers
// C = [A_np^T | A_pn] from its neighbour blocks using the current cluster
// sizes, runs the partial CPQR with FP64 norms and pivots, writes the coarse
// blocks back and stores the reflectors (column-major P x r, explicit unit
// diagonal and zeros above) and tau.  rank[cluster] receives r.
struct SpNbr {
  int64_t blk;      // element offset of block (i, p) or (p, j) in the interface's pool
  int32_t cluster;  // the neighbour cluster (its current size is rank[cluster])
  int32_t ld;       // leading dimension of the block
};

template <typename T>
struct SpDesc {
  T* C;             // P x mmax row-major workspace
  double* nrm;      // mmax doubles
  int32_t* perm;    // 2 * mmax ints
  T* vq;            // P x P column-major (first r columns used)
  T* tauq;          // P
  const int* flag;  // scaling flag of p (nonzero: not scaled, not sparsified)
  T* pool;          // block pool of the interface's factorization
  int* rank;        // current cluster sizes of that factorization (rank[cluster] gets r)
  double eps;       // truncation tolerance of that factorization
  int64_t nb;       // first neighbour in the SpNbr array
  int32_t nrow, ncol;
  int32_t cluster, P, mmax, pad;
};

// Sparsification without scaling (Section 2.5): one interface per workgroup.
constexpr int kSpuMaxP = 1024;   // largest interface
constexpr int kSpuMaxNbr = 512;  // most neighbour blocks of one interface
template <typename T>
struct SpuDesc {
  T* pool;        // block pool of the interface's factorization
  int* rank;      // current cluster sizes (rank[cluster] gets r)
  int* flag;      // set to 1 when p is left alone (sigma_min(A_p) = 0 or r = P)
  T* mf;          // P x P column-major forward operator Pi H^T
  T* mb;          // P x P column-major backward operator Q T
  double* ws;     // sparsify_unscaled_ws(P, mr_max, mc_max) doubles
  double eps;     // truncation tolerance
  int64_t app;    // element offset of the block (p, p) in the pool
  int64_t nb;     // first neighbour in the SpNbr array: nrow blocks (i, p), then ncol blocks (p, j)
  int32_t nrow, ncol;
  int32_t cluster, P;
  int32_t mr_max, mc_max;  // sums of the row / column neighbours' sizes at the start of the stage
};
int64_t sparsify_unscaled_ws(int P, int mr_max, int mc_max);
template <typename T>
void launch_sparsify_unscaled(const SpuDesc<T>* d, const SpNbr* nb, int64_t n, int max_p, hipStream_t s);

// Apply descriptors (vectors are FP64, slots index the permuted vector).
template <typename T>
struct ApFront {
  const T* vr;    // m x n column-major: V below the diagonal, R_ss on/above
  const T* rsj;   // n x k column-major
  const T* tau;   // n
  const T* tpan;  // compact-WY factor of every jb-reflector panel (jb x jb, column-major)
  const int32_t* rows;  // m slots: the front's row clusters
  const int32_t* cols;  // k slots: the ancestor column clusters
  int32_t m, n, k, jb;
  int32_t xoff;         // offset of the owning problem's vector in x (batched apply; 0 alone)
  int32_t pad;
};

template <typename T>
struct ApIface {
  const T* vru;   // P x P column-major scaling factor (U below diag, R_pp above)
  const T* tauu;
  const T* vq;    // P x P column-major sparsification reflectors (first r)
  const T* tauq;
  const int32_t* slots;  // P slots
  const int* rank;       // r (== P when nothing was dropped)
  const int* flag;       // nonzero: interface was not scaled
  T* mf;                 // P x P column-major Q^T U^T (P <= 64), formed after the stage
  T* mb;                 // P x P column-major R_pp^{-1} Q
  int32_t P;
  int32_t xoff;          // offset of the owning problem's vector in x (batched apply; 0 alone)
};

// ------------------------------------------------------------------ launchers
// Copy tiles, all transposing (transpose) or all plain.
template <typename T>
void launch_copy(const CopyTile<T>* tiles, int64_t ntiles, bool transpose, hipStream_t s);
template <typename T>
void launch_fill(T* p, int64_t n, T v, hipStream_t s);
template <typename T>
void launch_scatter_nz(T* pool, const int64_t* dst, const double* val, int64_t nnz, hipStream_t s);
void launch_colnorm(const int64_t* cptr, const int64_t* cidx, const double* val, int64_t n, double* dc,
                    int* zero_col, hipStream_t s);
template <typename T>
void launch_scatter_scaled(T* pool, const int64_t* dst, const double* val, const int32_t* col, const double* dc,
                           int64_t nnz, hipStream_t s);
// jb: panel width (power of two <= 32); lds_bytes: dynamic LDS per workgroup
template <typename T>
void launch_qr(const QRDesc<T>* d, int64_t n, int jb, int max_m, hipStream_t s);
// Trailing updates (TrailDesc).  trail_width: the slice width (16, 8 or 4
// columns) whose m x width slice fits LDS for fronts of at most max_m rows,
// 0 if none.  launch_trail: slices of at most cw columns, pivot blocks
// factored with panel width jb, at most max_m rows.
int trail_width(int max_m, int elem_bytes);
template <typename T>
void launch_trail(const TrailDesc<T>* d, int64_t n, int jb, int cw, int max_m, hipStream_t s);
// Matrix-core form of the trailing update: the T factors of every 64-reflector
// block, then the update of every 64-column tile.
constexpr int kWYBlock = 64;
template <typename T>
void launch_wy_tblock(const WYBlock<T>* d, int64_t n, hipStream_t s);
template <typename T>
void launch_trail_mfma(const WYTile<T>* d, int64_t n, hipStream_t s);
int qr_panel_width(int max_m, int elem_bytes);
size_t qr_lds_bytes(int max_m, int jb, int elem_bytes);
// Block scaling: B <- Q_i^T B R_j^{-1} (two launches); max_p bounds the
// interfaces' sizes (LDS panel of Q_i), max_rows / max_cols the blocks'.
template <typename T>
void launch_scale(const ScaleBlk<T>* d, int64_t n, const ScaleFac<T>* fac, int jb, int max_p, int max_rows,
                  int max_cols, hipStream_t s);
// The right factor alone (B <- B R_j^{-1}); identity blocks are left alone.
template <typename T>
void launch_scale_right(const ScaleBlk<T>* d, int64_t n, const ScaleFac<T>* fac, int max_rows, hipStream_t s);
// The same for blocks of at most kScaleSmall x kScaleSmall, one launch (the
// block staged in LDS once).
constexpr int kScaleSmall = 64;
template <typename T>
void launch_scale_small(const ScaleBlk<T>* d, int64_t n, const ScaleFac<T>* fac, int jb, int max_rows, int max_cols,
                        hipStream_t s);
// Zero fills; blocks = total workgroups (block0 of the last descriptor plus its own).
void launch_zero(const ZeroDesc* d, int64_t n, int64_t blocks, hipStream_t s);
constexpr int64_t kZeroWordsPerBlock = 4096;
template <typename T>
void launch_sparsify(const SpDesc<T>* d, int64_t n, const SpNbr* nb, int max_p, int max_nb, hipStream_t s);
// Interfaces of at most 64 unknowns; pmax = the largest P in the launch,
// max_c_elems = the largest P x m of the launch (C is staged in LDS when it fits).
// Register-resident CPQR (see k_cpqr_reg): columns per thread needed for
// interfaces of at most pmax unknowns and mmax columns, or 0 if they do not fit.
int sparsify_reg_cpt(int elem_bytes, int pmax, int mmax);
// whether that register CPQR also keeps a column per thread in the
// descriptor's workspace C (which then needs PMAX * 512 entries)
bool sparsify_reg_global(int elem_bytes, int pmax, int mmax);
template <typename T>
void launch_sparsify_reg(const SpDesc<T>* d, int64_t n, const SpNbr* nb, int pmax, int mmax, int max_nb,
                         hipStream_t s);
template <typename T>
void launch_sparsify_small(const SpDesc<T>* d, int64_t n, const SpNbr* nb, int pmax, int max_nb,
                           size_t max_c_elems, hipStream_t s);
// FP32 CPQR with downdated norms (k_cpqr_dd), every row class in one launch:
// the most columns an interface of P unknowns may have (0: P outside 1..64),
// and the LDS rows per thread a launch must provide for one of mmax columns
// (0: its columns fit in registers).  lc_rows = the largest of the launch.
int sparsify_dd_capacity(int P);
int sparsify_dd_lc_rows(int P, int mmax);
// A launch over several colours: workgroups take items in the order of the
// counter *ticket; item t first waits until done[pred[q]] != 0 for every q in
// [pred_ptr[t], pred_ptr[t + 1]) (all of them items before t: its adjacent
// interfaces of earlier colours), then, when succ[t] != 0 (some later item
// waits on it), sets done[t] once its results are visible device-wide.
// ticket and done[0 .. n) start at zero; *err is set when a bounded wait runs
// out.
struct DDFlow {
  int* ticket;
  int* done;
  const int* pred_ptr;
  const int* pred;
  const int* succ;
  int* err;
};
void launch_sparsify_dd(const SpDesc<float>* d, int64_t n, const SpNbr* nb, int max_nb, int lc_rows, hipStream_t s,
                        const DDFlow* flow = nullptr);
// Apply launches: max_rows = the largest number of FP64 rows one item keeps in
// LDS per right-hand side (m for fronts forward, n + k backward, P for
// interfaces).  Returns without launching when there is nothing to do.
int apply_rhs_block(int max_rows, int nrhs);
template <typename T>
void launch_front_fwd(const ApFront<T>* d, int64_t n, int max_rows, double* x, int64_t ldx, int nrhs, hipStream_t s);
// Panel-blocked forward sweep: every front of the launch has panel width jb.
template <typename T>
void launch_front_fwd_wy(const ApFront<T>* d, int64_t n, int jb, int max_rows, double* x, int64_t ldx, int nrhs,
                         hipStream_t s);
// Backward sweep with register-accumulated R_sj products; max_n <= 1024.
template <typename T>
void launch_front_bwd_reg(const ApFront<T>* d, int64_t n, int max_n, int max_k, double* x, int64_t ldx, int nrhs,
                          hipStream_t s);
// Interfaces of at most 64 unknowns: one wavefront, one row per lane.
// Cooperative CPQR for interfaces too large for one workgroup: interface i
// owns workgroups [first, first + nblk) of one cooperative launch (64 threads
// each, 64 * cpt columns per workgroup); C lives row-major in the
// interface's workspace (d.C, leading dimension d.mmax).
struct CoopItem {
  int32_t first, nblk;
};
// FP32 CPQR of wide interfaces by teams of co-resident workgroups
// (k_cpqr_team): workgroups a team needs for P unknowns and mmax columns (0:
// P outside 1..896), workgroups one launch may hold, the bytes of the
// candidate buffer for launches of at most max_blocks workgroups, and the
// launch.  items: each team's first workgroup and size; sync: two zeroed ints
// per team (left zeroed for reuse); cand: the candidate buffer, laid out for
// cand_blocks workgroups; err: set to 1 if a team barrier wait ran out (the
// kernel then still ends, with invalid results).  Returns false (nothing
// launched) when the workgroups cannot be co-resident.
int sparsify_team_blocks(int P, int mmax);
int sparsify_team_capacity(int max_nb);
size_t sparsify_team_cand_bytes(int max_blocks);
bool launch_sparsify_team(const SpDesc<float>* d, const CoopItem* items, int nitems, int total_blocks,
                          const SpNbr* nb, int max_nb, int* sync, void* cand, int cand_blocks, int* err,
                          hipStream_t s);
// Returns false (nothing launched) if the items cannot be co-resident; then
// the caller falls back to the single-workgroup kernels.
template <typename T>
bool launch_sparsify_coop(const SpDesc<T>* d, const CoopItem* items, int nitems, int total_blocks, int cpt,
                          const SpNbr* nb, int max_p, int max_nb, double* ckey, int* cpos, T* ccol, int* done,
                          int kmax_all, hipStream_t s);
// Largest number of one-wave workgroups that can be co-resident for the
// cooperative CPQR with columns-per-thread cpt and rows max_p.
template <typename T>
int sparsify_coop_capacity(int cpt, int max_p, int max_nb);

// Dense interface operators (P <= 64): mf = Q^T U^T and mb = R_pp^{-1} Q,
// one thread per column; then the apply multiplies by them.
template <typename T>
void launch_iface_form(const ApIface<T>* d, int64_t n, int max_p, hipStream_t s);  // max_p <= 64
template <typename T>
void launch_iface_dense(const ApIface<T>* d, int64_t n, bool backward, double* x, int64_t ldx, int nrhs,
                        hipStream_t s, int max_p);
// the same for interfaces of any size up to kSpuMaxP, one workgroup each
template <typename T>
void launch_iface_dense_big(const ApIface<T>* d, int64_t n, bool backward, double* x, int64_t ldx, int nrhs,
                            hipStream_t s);
template <typename T>
void launch_iface_small(const ApIface<T>* d, int64_t n, bool backward, double* x, int64_t ldx, int nrhs,
                        hipStream_t s);
template <typename T>
void launch_front_bwd(const ApFront<T>* d, int64_t n, int max_rows, double* x, int64_t ldx, int nrhs, hipStream_t s);
template <typename T>
void launch_iface_fwd(const ApIface<T>* d, int64_t n, int max_rows, double* x, int64_t ldx, int nrhs, hipStream_t s);
template <typename T>
void launch_iface_bwd(const ApIface<T>* d, int64_t n, int max_rows, double* x, int64_t ldx, int nrhs, hipStream_t s);
// xhat[i + c*N] = b[perm[i] + c*ldb]
void launch_gather_perm(double* xhat, const double* b, int64_t ldb, const int64_t* perm, int64_t N,
                        int nrhs, hipStream_t s);
// x[perm[i] + c*ldx] = xhat[i + c*N] * dc[perm[i]]
void launch_scatter_perm(double* x, int64_t ldx, const double* xhat, const int64_t* perm,
                         const double* dc, int64_t N, int nrhs, hipStream_t s);

// One column of an apply batched across problems: column col of b and x; its
// problem has n unknowns, permutation perm and column scaling dc; its
// permuted vector lives at xhat + xoff.
struct PermCol {
  int64_t col, xoff;
  const int64_t* perm;
  const double* dc;
  int64_t n;
};
// out[op.dst + i] = op.src[i] for i < op.n, for every op of the list
struct IntCopy {
  const int32_t* src;
  int32_t dst, n;
};
void launch_gather_ints(const IntCopy* ops, int nops, int32_t* out, hipStream_t s);
// xhat[pc[j].xoff + i] = b[pc[j].perm[i] + pc[j].col*ldb] for every j < ncols
void launch_gather_cols(double* xhat, const double* b, int64_t ldb, const PermCol* pc, int ncols, int64_t max_n,
                        hipStream_t s);
// x[pc[j].perm[i] + pc[j].col*ldx] = xhat[pc[j].xoff + i] * pc[j].dc[pc[j].perm[i]]
void launch_scatter_cols(double* x, int64_t ldx, const double* xhat, const PermCol* pc, int ncols, int64_t max_n,
                         hipStream_t s);

// CSR matrix of one column of a batched SpMV.
struct SpmvCol {
  const int64_t* rowptr;
  const int32_t* col;
  const double* val;
  int64_t n;
};
// y[:, j] = A_j x[:, j] over the first sc[j].n rows (the rest untouched)
void launch_spmv_cols(const SpmvCol* sc, int ncols, int64_t max_n, const double* x, int64_t ldx, double* y,
                      int64_t ldy, hipStream_t s);

}  // namespace spaqr
