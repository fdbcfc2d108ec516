// Device operations used by the RT-EOM-CCSD engine.
//
// The engine (engine.cpp) expresses one residual evaluation and one time step
// as a sequence of these operations; backend_hip.hip implements them with
// hand-written gfx950 kernels.  Complex tensors are planar: a real plane and an
// imaginary plane with identical strides.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

namespace rteom {

constexpr int kMaxDims = 6;

// C[b](m, n) = alpha * sum_k A[b](m, k) * B[b](k, n) + beta * C[b](m, n)
// Each operand element is at base + b*sb + i*s0 + j*s1.  An operand whose
// imaginary pointer is null is real.  C is real exactly when A and B are real.
struct GemmOp {
  int64_t M = 0, N = 0, K = 0, batch = 1;
  const double* a_re = nullptr; const double* a_im = nullptr; int64_t a_sm = 0, a_sk = 0, a_sb = 0;
  const double* b_re = nullptr; const double* b_im = nullptr; int64_t b_sk = 0, b_sn = 0, b_sb = 0;
  double* c_re = nullptr; double* c_im = nullptr; int64_t c_sm = 0, c_sn = 0, c_sb = 0;
  double alpha = 1.0;
  int beta = 0;      // 0 overwrite, 1 accumulate
  int prec = 0;      // rteom_prec
  // split-K (batch == 1 only): the K range is cut into `splitk` chunks whose
  // partial products go to `partial` ([splitk][M][N], planar when complex) and
  // are summed in a fixed order by a second kernel.
  int splitk = 1;
  double* partial = nullptr;
  // Operands converted once before the product (reduced precisions): scratch of
  // split_doubles(...) doubles that receives A and B in the contraction's storage
  // ([batch][rows][k], k contiguous, zero padded to kSplitK; one matrix when the
  // operand's batch stride is 0): bf16 hi/lo planes
  // for bf16x3, float planes for fp32.  nullptr = convert while staging.
  double* split = nullptr;
  // A real B held converted outside the scratch (a constant operand): its planes
  // ([N][ld], the layout the conversion above gives B) are at b_conv; with
  // b_conv_fill = 1 this product converts B into them first, else it reads them
  // as they are.  The scratch then holds A's planes only.
  double* b_conv = nullptr;
  int b_conv_fill = 0;
};

// K granularity of converted planes, and the scratch (in doubles) they need.
constexpr int64_t kSplitK = 32;
inline int64_t split_ld(int64_t K) { return (K + kSplitK - 1) / kSplitK * kSplitK; }
// batch_a / batch_b: matrices of each operand (1 when it is the same for every batch entry)
inline int64_t split_doubles(int64_t M, int64_t N, int64_t K, int64_t batch_a, int64_t batch_b, bool ac, bool bc,
                             int prec) {
  // elements of all real planes of A ([M][ld]) and B ([N][ld])
  const int64_t el = split_ld(K) * (batch_a * M * (ac ? 2 : 1) + batch_b * N * (bc ? 2 : 1));
  // bf16x3 / fp16x3: two 2-byte planes per real plane; fp32: one 4-byte plane; +64 for
  // alignment.  fp16x3 adds each row's maximum and inverse scale (4 bytes each).
  const int64_t scales = prec == 3 ? batch_a * M + batch_b * N : 0;
  return (prec >= 2 ? (2 * el + 3) / 4 : (el + 1) / 2) + scales + 64;
}

// Doubles that hold one real operand of `rows` rows converted for a sum of K: two
// bf16 planes or one float plane, [rows][split_ld(K)] each (+64 for alignment).
inline int64_t conv_doubles(int64_t rows, int64_t K) { return (rows * split_ld(K) + 1) / 2 + 64; }

// out[idx] = alpha * in[idx] * prod_d scale_d[idx_d] + beta * out[idx] over an
// nd-dimensional index space; strides per operand.  in may be real while out is
// complex (then alpha may be complex).  in == out with beta = 0 scales in place.
// alpha = 0 with beta = 0 writes zeros (whatever in holds).
struct PermOp {
  int nd = 0;
  int64_t dim[kMaxDims] = {0};
  const double* in_re = nullptr; const double* in_im = nullptr; int64_t in_str[kMaxDims] = {0};
  double* out_re = nullptr; double* out_im = nullptr; int64_t out_str[kMaxDims] = {0};
  const double* scale[kMaxDims] = {nullptr};  // optional real vector per dimension
  double alpha_re = 1.0, alpha_im = 0.0;
  int beta = 0;
};

// Index pairs i < j of n indices in lexicographic order: pair (i, j) is number
// pair_start(i, n) + j - i - 1.
inline int64_t npairs(int64_t n) { return n * (n - 1) / 2; }
inline int64_t pair_start(int64_t i, int64_t n) { return i * (2 * n - i - 1) / 2; }

// Layout of an amplitude set, planar (all real parts, then all imaginary parts):
//   t1 alpha [no][nv], t1 beta [no][nv],
//   t2 alpha-alpha [npairs(no)][npairs(nv)]  (t_ijab for i < j, a < b),
//   t2 beta-beta   [npairs(no)][npairs(nv)],
//   t2 alpha-beta  [no][no][nv][nv].
// The same-spin doubles are antisymmetric in (i, j) and in (a, b); only their
// unique elements are stored.
struct AmpLayout {
  int64_t no = 0, nv = 0;
  int64_t n1() const { return no * nv; }
  int64_t npo() const { return npairs(no); }
  int64_t npv() const { return npairs(nv); }
  int64_t nss() const { return npo() * npv(); }          // one same-spin block
  int64_t nab() const { return no * no * nv * nv; }      // the alpha-beta block
  int64_t off_ss(int s) const { return 2 * n1() + s * nss(); }
  int64_t off_ab() const { return 2 * n1() + 2 * nss(); }
  int64_t size() const { return 2 * n1() + 2 * nss() + nab(); }
};

// Pair tables on the device: for pair p, first[p] < second[p] (int32).
struct PairTables {
  const int32_t* oi = nullptr; const int32_t* oj = nullptr;   // occupied pairs, [npairs(no)]
  const int32_t* va = nullptr; const int32_t* vb = nullptr;   // virtual pairs, [npairs(nv)]
};

// Per-spin occupancy masks and Fock diagonals (device vectors), used to zero
// amplitudes of non-existent spin-orbitals and by the diagonal map.
struct SpinVectors {
  const double* mo[2] = {nullptr, nullptr};  // [no]
  const double* mv[2] = {nullptr, nullptr};  // [nv]
  const double* fo[2] = {nullptr, nullptr};  // [no] f_ii
  const double* fv[2] = {nullptr, nullptr};  // [nv] f_aa
};

// Fused amplitude update of Eq. trapzrule (see engine.cpp, step()):
//   start: rhs = x + i h r; then for every amplitude
//   plain:       x' = rhs + i h r
//   denominator: x' = (rhs + i h (r + D x)) / (1 + i h D)
//   Jacobi:      x' = x + r / D   (mode 2, ground state R(T) = 0; rhs unused)
//   x' = 0 where the spin-orbital does not exist;  *delta = max |x' - x|.
struct UpdateOp {
  AmpLayout lay;
  PairTables pt;
  double* x_re = nullptr; double* x_im = nullptr;
  const double* r_re = nullptr; const double* r_im = nullptr;
  double* rhs_re = nullptr; double* rhs_im = nullptr;
  double h = 0.0;      // dt / 2
  int mode = 0;        // 0 plain, 1 denominator, 2 Jacobi
  int start = 0;       // 1: form rhs from x and r first (stored when rhs_re is set)
  SpinVectors sv;
  double* delta = nullptr;  // device double, max-reduced (caller zeroes it)
};

// Same-spin doubles between antisymmetric pair storage y [npairs(n1)][npairs(n2)] (planar
// complex when y_im is set, else real) and full storage.  x is a block of a full tensor
// [n1][n1][n2][n2] holding rows i0 .. i0+ci-1 and columns j0 .. j0+cj-1 of the first two
// indices, row-major [ci][cj][n2][n2] (x_im with y_im).
//   kExpand:     x[i][j][a][b] = alpha s y[pair(i,j)][pair(a,b)] + beta x  (s = -1 per
//                swapped pair; 0 where i = j or a = b)
//   kAccum:      y[pair(i,j)][pair(a,b)] += alpha (sum over the block's elements that map
//                there): the antisymmetric part of x -- with anti1 the element (i,j) adds
//                to pair (i,j) and with a minus sign to pair (j,i) (P(ij)); without it x
//                is antisymmetric in (i,j) already and only i < j is read.  anti2 likewise
//                for (a,b).  Every pair is written by one thread (no atomics).
//   kAccumRows:  x is [cp][n2][n2] over pairs p0 .. p0+cp-1 of the first index:
//                y[p][pair(a,b)] += alpha (x[p][a][b] - anti2 x[p][b][a])
//   kT1T1:       y[p][q] = beta y + alpha (u_ia u_jb - u_ib u_ja), u = [n1][n2] complex
//                (u_re/u_im), (i,j) = pair p, (a,b) = pair q
//   kMask:       y[p][q] *= m1[i] m1[j] m2[a] m2[b]
//   kPackSlab:   integral slab x [ce][n1][rest] holding rows e0 .. e0+ce-1 of a real
//                [n1][n1][rest] tensor (rest = n2 n2 with pair2, else n2); y gets the
//                pairs (e < f) with e in the slab, in order, rows [npairs-range][nq]:
//                pair2: y[.][pair(a,b)] = alpha (x[e][f][a][b] - x[e][f][b][a]),
//                else   y[.][c] = alpha x[e][f][c].
struct SsOp {
  enum Mode { kExpand = 0, kAccum = 1, kAccumRows = 2, kT1T1 = 3, kMask = 4, kPackSlab = 5 };
  int mode = 0;
  int64_t n1 = 0, n2 = 0;
  int64_t i0 = 0, ci = 0, j0 = 0, cj = 0;   // block of x (kExpand, kAccum); p0, cp in i0, ci for kAccumRows;
                                            // e0, ce in i0, ci for kPackSlab
  int pair2 = 1;
  int anti1 = 1, anti2 = 1;
  double alpha = 1.0;
  int beta = 0;
  double* x_re = nullptr; double* x_im = nullptr;
  double* y_re = nullptr; double* y_im = nullptr;
  const double* u_re = nullptr; const double* u_im = nullptr;
  const double* m1 = nullptr; const double* m2 = nullptr;
  PairTables pt;   // tables of n1 (oi/oj) and n2 (va/vb) pairs
};

// E(T) = sum f_ia t_ia + 1/4 sum <ij||ab> t_ijab + 1/2 sum <ij||ab> t_ia t_jb in
// spin-blocked form; writes (re, im) to e_out (device).
struct EnergyOp {
  AmpLayout lay;
  const double* x_re = nullptr; const double* x_im = nullptr;
  const double* jov = nullptr;        // (ia|jb) as [i][a][j][b]
  const double* fov[2] = {nullptr, nullptr};  // f^s_ia as [no][nv] (row stride fov_ld)
  int64_t fov_ld = 0;
  int include_ft1 = 1;
  double* e_out = nullptr;
  double* partial = nullptr;          // scratch, >= energy_partials() doubles
};

// Phases of one residual evaluation / time step; device timing can be switched
// on per phase (HIP events around each operation of a selected phase only).
enum Phase {
  kPhaseLadder = 0,   // particle-particle ladder GEMM
  kPhaseRing = 1,     // o^3 v^3 ring / W / Z GEMMs
  kPhaseGemm = 2,     // all other GEMMs
  kPhaseMove = 3,     // permutes, copies, scaling
  kPhaseUpdate = 4,   // fused trapezoid update
  kPhaseEnergy = 5,   // energy reduction and C(t) append
  kPhaseBuild = 6,    // integral slabs rebuilt from the Cholesky vectors
  kNumPhases = 7
};

class Backend {
 public:
  virtual ~Backend() {}
  virtual void set_phase(int ph) { phase_ = ph; }
  virtual void set_profile(unsigned mask) { (void)mask; }
  // GEMM tile shape: 1 = time the candidates the first time a shape is met
  // (outside capture) and keep the fastest, 0 = work-per-byte rule.
  virtual void set_tuning(int on) { (void)on; }
  // Test hook: force one tile shape (0: 64x64, 1: 64x128, 2: 128x64,
  // 3: 128x128, 4: 64x128 and 5: 128x64 with eight waves) where the operand
  // types and precision allow it (else 64x64); -1 = automatic.
  virtual void force_tile(int v) { (void)v; }
  // Timed tile choices, kTileKey + 1 values per entry (the GEMM signature, then the tile
  // shape): tile_table copies up to max entries into rows and returns how many there are;
  // load_tile_table adds entries (a later entry for the same signature replaces it) and
  // rejects a table whose tile shape is not built for its signature.
  static constexpr int kTileKey = 10;
  virtual int64_t tile_table(int64_t* rows, int64_t max) const { (void)rows; (void)max; return 0; }
  virtual bool load_tile_table(const int64_t* rows, int64_t n, std::string* err) {
    (void)rows;
    if (n > 0 && err) *err = "this backend keeps no tile choices";
    return n == 0;
  }
  // the device's architecture name (tile choices are only valid on it)
  virtual std::string device_arch() const { return "host"; }
  // total milliseconds and operation count of the profiled phase since the last call
  virtual double phase_ms(int ph, int64_t* ops) { (void)ph; if (ops) *ops = 0; return 0.0; }
 protected:
  int phase_ = kPhaseGemm;
 public:
  virtual void* alloc(size_t bytes) = 0;
  virtual void release(void* p) = 0;
  virtual void h2d(void* dst, const void* src, size_t bytes) = 0;
  virtual void d2h(void* dst, const void* src, size_t bytes) = 0;   // synchronous
  virtual void d2d(void* dst, const void* src, size_t bytes) = 0;
  virtual void fill(double* p, int64_t n, double v) = 0;
  virtual void gemm(const GemmOp& op) = 0;
  virtual void permute(const PermOp& op) = 0;
  virtual void ss(const SsOp& op) = 0;
  virtual void update(const UpdateOp& op) = 0;
  virtual void energy(const EnergyOp& op) = 0;
  // With k = *step (device): C[k+1] = C[k] + i h (E[k] + e_next), E[k+1] = e_next,
  // *step = k + 1.  c_hist, e_hist: device (re, im) pairs; e_next: device pair.
  // *bad (device) becomes 1 if e_next or C[k+1] is not finite and is never cleared
  // here: E(T) sums every amplitude times an integral, so it is NaN or infinite as
  // soon as one amplitude is.
  virtual void cumulant_append(double* c_hist, double* e_hist, const double* e_next,
                               int64_t* step, double h, double* bad) = 0;
  // *out = sum_k a[k] b[k] (device pointers), summed in a fixed order; part is
  // scratch of energy_partials() doubles.
  virtual void dot(const double* a, const double* b, int64_t n, double* part, double* out) = 0;
  // Spectral function from the cumulant history (all pointers device memory):
  // c_hist [n][2] C(t_k), times [n], omega [n_w] -> a_out [n_w] A(omega),
  // qp_out [2] = (refined position of the largest A, A at the grid maximum);
  // shift = eps_c + E_N^corr, eta = damping; wg is scratch of 2 n doubles.
  virtual void spectral(const double* c_hist, const double* times, int64_t n, double shift, double eta,
                        const double* omega, int64_t n_w, double* wg, double* a_out, double* qp_out) = 0;
  // Peaks of a spectrum a [n_w] on the uniform grid omega (device pointers): the local maxima
  // (a[j] > a[j-1] and a[j] >= a[j+1], 0 < j < n_w - 1), the largest first (first index on
  // ties), at most k of them; out [k][2] = (position refined by the parabola through the
  // maximum and its neighbours, a[j]), out[2k] = number found.
  virtual void spectral_peaks(const double* a, const double* omega, int64_t n_w, int k, double* out) = 0;
  // Stream capture of a fixed sequence of operations into a replayable graph
  // (returns false where not supported: the caller then issues operations directly).
  virtual bool begin_capture() { return false; }
  virtual bool capturing() const { return false; }
  virtual void* end_capture() { return nullptr; }
  virtual void launch_graph(void* exec) { (void)exec; }
  virtual void destroy_graph(void* exec) { (void)exec; }
  virtual void* stream() { return nullptr; }
  // Device memory of a fixed size that needs no allocation (nullptr where there is
  // none); *doubles receives its capacity.  Shared by every caller on the device.
  virtual double* fixed_scratch(int64_t* doubles) { if (doubles) *doubles = 0; return nullptr; }
  virtual int64_t energy_partials() const = 0;
  virtual void sync() = 0;
  // returns false (and a message) if an asynchronous error has been recorded
  virtual bool ok(std::string* msg) = 0;
};

Backend* make_hip_backend(void* stream, std::string* err);

}  // namespace rteom
