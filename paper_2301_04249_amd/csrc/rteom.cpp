// RT-EOM-CCSD propagation context and the C ABI (include/rteom.h).
//
// Formulation (what the device computes; arXiv 2301.04249, Sec. 2.1 and 3):
//
// * Reference.  |Phi> is the N-electron determinant with spin-orbital c removed.
//   All quantities live in an "extended" orbital space O + V, where O holds the
//   orbitals occupied in Phi in either spin and V the orbitals virtual in either
//   spin; per-spin masks zero the amplitudes of spin-orbitals that do not exist
//   (for a beta hole: beta amplitudes with occupied index c, alpha amplitudes
//   with virtual index c).  Integrals are spin free, so all three T2 blocks
//   (aa, ab, bb) share one set of integral blocks.  The same-spin doubles are
//   stored over their unique pairs (i < j, a < b); the alpha-beta block in full.
// * Residual.  R_x = <Phi_x| e^{-T} H_N e^{T} |Phi> is evaluated in the
//   T1-similarity-transformed ("dressed") form: e^{-T1} H e^{T1} has the
//   Cholesky vectors L~ = (1 - t) L (1 + t) (t: the virtual-by-occupied T1
//   matrix) and the dressed Fock matrix f~ = (1 - t) h (1 + t) + J~ - K~ of Phi,
//   and R is the CCD-like projection of that Hamiltonian with T2 (Eqs. dt1eom,
//   dt2eom).  The pp-ladder keeps the real (ae|bf) integrals; the T1 part of the
//   dressed virtual vectors becomes the o^3 v^3 "Z" terms and an o^4 v^2 term.
//   Coulomb-type ring terms are factorised through D^Q_ia = sum_me T_imae L^Q_me.
// * Memory.  Every intermediate that grows like o^2 v^2 or faster is produced in
//   blocks when the whole would not fit: the ring intermediates W[(m,e),(b,j)] in
//   blocks of j, expanded same-spin amplitudes in blocks of rows, and -- when they
//   cannot stay resident -- (ae|bf), (me|bf) and their pair forms rebuilt from the
//   Cholesky vectors in slabs of e for every residual.  A plan chosen at init
//   (the largest blocks that keep the workspace within the memory limit) fixes
//   the block sizes; the arithmetic of every element is the same for any plan.
// * Step.  Implicit trapezoid (Eq. trapzrule) with fixed-point passes; three
//   amplitude-sized buffers (iterate X, rhs, residual R) as in Table 2's three
//   timeline tensors.  C(t) accumulates i E(T) with the same trapezoid weights.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rteom.h"
#include "backend.h"
#include "engine.h"

namespace rteom {

Backend* make_host_backend();

// Largest GEMM-order temporary of the integral-block build (2 GiB of doubles).
constexpr int64_t kSlabDoubles = int64_t(1) << 28;
// Default memory limit of the plan: MI355X HBM (288 GiB) less room for the runtime.
constexpr size_t kDefaultMemLimit = size_t(270) << 30;
// Rows of packed same-spin pairs per block of the Z-term expansion.
constexpr int64_t kPairRowDoubles = int64_t(1) << 28;

// Block sizes of one residual evaluation (see "Memory" above).
struct Plan {
  bool resident = true;   // (ae|bf), (me|bf) and their same-spin pair forms built once at init
  int64_t es = 0;         // else rebuilt per residual in slabs of es virtual indices e
  int64_t cj = 0;         // occupied columns j per block of the ring intermediates
  int64_t ci = 0;         // occupied rows per block of expanded same-spin amplitudes
};

struct Context {
  rteom_options opt{};
  Backend* be = nullptr;
  bool dry = false;
  Arena arena;
  Engine eng;
  void* ws = nullptr;
  bool ws_owned = false;
  std::string err;
  bool failed = false;
  Plan plan;

  int n = 0, nq = 0, na = 0, nb = 0, core_orb = 0, core_spin = 0;
  int no = 0, nv = 0, nx = 0;
  std::vector<int> O, V;
  std::vector<double> mo_h[2], mv_h[2];
  AmpLayout lay;
  // fractions of existing spin-orbitals per extended index range (flop accounting)
  double f_o[2] = {1, 1}, f_v[2] = {1, 1}, f_po[2] = {1, 1}, f_pv[2] = {1, 1};

  double* mo[2] = {nullptr, nullptr};
  double* mv[2] = {nullptr, nullptr};
  double* fo[2] = {nullptr, nullptr};
  double* fv[2] = {nullptr, nullptr};
  int32_t* ptab = nullptr;             // pair tables: occupied (i, j), virtual (a, b)
  double *Loo = nullptr, *Lov = nullptr, *Lvv = nullptr, *Lvo = nullptr;
  double* f[2] = {nullptr, nullptr};   // undressed Fock of Phi, [nx][nx]
  double* h[2] = {nullptr, nullptr};   // one-body part h = f - G, [nx][nx]
  double* Jov = nullptr;               // (me|nf) as [m][e][n][f]
  double* Jx = nullptr;                // (mf|ne) as [n][f][m][e]: the ring intermediates' exchange operand
  double* Jp = nullptr;                // (me|nf) - (mf|ne) as [e<f][m<n]
  // Resident plan only: (ae|bf) as [e][f][a][b], (me|bf) as [e][f][m][b], and the
  // same-spin pair forms <ab||ef> = (ae|bf) - (af|be) as [e<f][a<b] and
  // (me|bf) - (mf|be) as [e<f][m][b]
  double* Vlad = nullptr;
  double* B1 = nullptr;
  double* Wpp = nullptr;
  double* B1p = nullptr;
  // reduced precisions: the contractions' converted copies of those constant blocks
  // (ladder, same-spin ladder, alpha-beta Z, same-spin Z), made by their first use
  ConvSlot conv_v, conv_w, conv_b1, conv_b1p;
  double *X = nullptr, *RHS = nullptr, *R = nullptr;   // amplitude sets
  double* Tn = nullptr;      // T_n kept by tolerance-driven steps (restored if a step fails)
  bool restored = false;     // the last failed step left T and C(t) as they were
  double* delta = nullptr;
  double* dbad = nullptr;    // device flag: a non-finite E(T) or C(t) was appended
  double* epart = nullptr;
  double* e_hist = nullptr;  // [(max_steps+1)][2]
  double* e_next = nullptr;  // E(T_{n+1}) of the step in flight
  // Anderson acceleration of the tolerance-driven fixed points: ring of the last
  // am iterates x_j and differences f_j = G(x_j) - x_j, their Gram matrix (host)
  int am = 0, a_count = 0, a_head = 0;
  std::vector<double*> a_x, a_f;
  std::vector<double> a_gram;
  double* a_dot = nullptr;
  int64_t* dstep = nullptr;  // steps taken, on the device (indexes the histories)
  void* step_graph = nullptr;
  double graph_dt = 0.0;
  double* c_hist = nullptr;  // [(max_steps+1)][2]
  int64_t nsteps = 0;
  std::vector<double> times;
  double eps_core = 0.0;               // N-electron orbital energy of the ionised orbital
  double res_flops = 0.0, res_alg_flops = 0.0;
  double res_phase_flops[kNumPhases] = {0}, res_alg_phase_flops[kNumPhases] = {0};

  // ---------------------------------------------------------------- views
  int64_t npo() const { return lay.npo(); }
  int64_t npv() const { return lay.npv(); }
  View Lv(double* p, int64_t a, int64_t b) const { return make_view(p, nullptr, {nq, a, b}); }
  View t1(double* set, int s) const {
    return with_frac(make_view(set + s * lay.n1(), set + lay.size() + s * lay.n1(), {no, nv}), {f_o[s], f_v[s]});
  }
  // alpha-beta doubles t_{i alpha, j beta}^{a alpha, b beta} as [i][j][a][b]
  View tab(double* set) const {
    double* p = set + lay.off_ab();
    return with_frac(make_view(p, p + lay.size(), {no, no, nv, nv}), {f_o[0], f_o[1], f_v[0], f_v[1]});
  }
  // the same rows as [(i,j)][e][f]
  View tab3(double* set) const {
    double* p = set + lay.off_ab();
    return with_frac(make_view(p, p + lay.size(), {(int64_t)no * no, nv, nv}), {f_o[0] * f_o[1], f_v[0], f_v[1]});
  }
  // t_{i s, m u}^{a s, e u} for s != u as [i][m][a][e]
  View tsu(double* set, int s) const { return s == 0 ? tab(set) : reorder(tab(set), {1, 0, 3, 2}); }
  // same-spin block s in pair storage [i<j][a<b]
  View tss(double* set, int s) const {
    double* p = set + lay.off_ss(s);
    return with_frac(make_view(p, p + lay.size(), {npo(), npv()}), {f_po[s], f_pv[s]});
  }
  // both same-spin blocks as one [(s, i<j)][a<b]
  View tss2(double* set) const {
    double* p = set + lay.off_ss(0);
    return with_frac(make_view(p, p + lay.size(), {2 * npo(), npv()}),
                     {0.5 * (f_po[0] + f_po[1]), 0.5 * (f_pv[0] + f_pv[1])});
  }
  View fview(double* p, int64_t r0, int64_t c0, int64_t nr, int64_t nc, bool cplx) const {
    View v = make_view(p, cplx ? p + (int64_t)nx * nx : nullptr, {nx, nx});
    return block(v, {r0, c0}, {nr, nc});
  }
  View vec(double* p, int64_t n) const { return make_view(p, nullptr, {n}); }
  PairTables tables() const {
    PairTables t;
    t.oi = ptab;
    t.oj = ptab + npo();
    t.va = ptab + 2 * npo();
    t.vb = ptab + 2 * npo() + npv();
    return t;
  }
  SsOp ss_op(int mode, double* set, int s) const {
    SsOp op;
    op.mode = mode;
    op.n1 = no;
    op.n2 = nv;
    op.y_re = set + lay.off_ss(s);
    op.y_im = set + lay.size() + lay.off_ss(s);
    op.pt = tables();
    return op;
  }
  // Rows i0 .. i0+ci-1 (all j) of same-spin block s, expanded to full storage [ci][no][nv][nv].
  View expand_rows(double* set, int s, int64_t i0, int64_t ci) {
    View x = eng.temp({ci, no, nv, nv}, true);
    SsOp op = ss_op(SsOp::kExpand, set, s);
    op.i0 = i0; op.ci = ci; op.j0 = 0; op.cj = no;
    op.x_re = x.re; op.x_im = x.im;
    eng.ss(op);
    return with_frac(x, {f_o[s], f_o[s], f_v[s], f_v[s]});
  }
  // Same-spin block s of set += alpha * (antisymmetric part of) the block x of rows i0..,
  // columns j0.. (SsOp::kAccum).
  void accum(double* set, int s, const View& x, int64_t i0, int64_t j0, double alpha, int anti1, int anti2) {
    SsOp op = ss_op(SsOp::kAccum, set, s);
    op.i0 = i0; op.ci = x.dim[0]; op.j0 = j0; op.cj = x.dim[1];
    op.x_re = x.re; op.x_im = x.im;
    op.alpha = alpha; op.anti1 = anti1; op.anti2 = anti2;
    eng.ss(op);
  }
  View sstemp(std::initializer_list<int64_t> dims, int s) {
    View x = eng.temp(dims, true);
    return with_frac(x, {f_o[s], f_o[s], f_v[s], f_v[s]});
  }

  // Progress report of a long residual evaluation (rteom_options.progress): waits for the
  // stream, then one line to stderr.
  std::chrono::steady_clock::time_point t_res;
  void progress(const char* what, int64_t k, int64_t n) {
    if (dry || !opt.progress) return;
    be->sync();
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_res).count();
    std::fprintf(stderr, "[rteom] residual: %s %lld/%lld done (%.1f s)\n", what, (long long)k, (long long)n, s);
    std::fflush(stderr);
  }

  double* take(int64_t n) { return arena.take(n); }
  void h2d(double* dst, const double* src, int64_t n) {
    if (!dry) be->h2d(dst, src, n * sizeof(double));
  }
  void fill(double* p, int64_t n) {
    if (!dry) be->fill(p, n, 0.0);
  }
  void check() {
    if (dry) return;
    std::string m;
    if (!be->ok(&m)) throw Error(RTEOM_ERR_HIP, m);
  }

  // ------------------------------------------------------------ set-up
  void setup_spaces() {
    std::vector<char> occ[2], vir[2];
    for (int s = 0; s < 2; ++s) {
      occ[s].assign(n, 0);
      int ns = s == 0 ? na : nb;
      for (int p = 0; p < ns; ++p) occ[s][p] = 1;
    }
    if (core_orb >= 0) occ[core_spin][core_orb] = 0;   // core_orb < 0: the N-electron determinant
    for (int s = 0; s < 2; ++s) {
      vir[s].assign(n, 0);
      for (int p = 0; p < n; ++p) vir[s][p] = !occ[s][p];
    }
    O.clear();
    V.clear();
    for (int p = 0; p < n; ++p) {
      if (occ[0][p] || occ[1][p]) O.push_back(p);
      if (vir[0][p] || vir[1][p]) V.push_back(p);
    }
    no = (int)O.size();
    nv = (int)V.size();
    nx = no + nv;
    for (int s = 0; s < 2; ++s) {
      mo_h[s].resize(no);
      mv_h[s].resize(nv);
      int cnt_o = 0, cnt_v = 0;
      for (int i = 0; i < no; ++i) cnt_o += (mo_h[s][i] = occ[s][O[i]]) != 0;
      for (int a = 0; a < nv; ++a) cnt_v += (mv_h[s][a] = vir[s][V[a]]) != 0;
      f_o[s] = no ? (double)cnt_o / no : 1.0;
      f_v[s] = nv ? (double)cnt_v / nv : 1.0;
      f_po[s] = npairs(no) ? (double)npairs(cnt_o) / npairs(no) : 1.0;
      f_pv[s] = npairs(nv) ? (double)npairs(cnt_v) / npairs(nv) : 1.0;
    }
    lay.no = no;
    lay.nv = nv;
  }

  // (ae|bf) [ce][nv][nv][nv], <ab||ef> rows [pairs (e<f), e in slab][a<b], (me|bf)
  // [ce][nv][no][nv] and (me|bf) - (mf|be) rows [pairs (e<f), e in slab][m][b] for the
  // virtual indices e0 .. e0+ce-1 (Sec. 2.3: (pq|rs) = sum_Q L^Q_pq L^Q_rs), in the
  // engine's current precision.
  // Cholesky vectors with the vector index Q innermost, the operand layout of the slab
  // products (both operands then stream along their sum index): Lt_vv[p][q][Q] over
  // virtual p, q and Lt_vo[e][m][Q] = L^Q_me.
  struct SlabOperands {
    View vv, vo;
  };
  SlabOperands slab_operands() {
    SlabOperands o;
    o.vv = eng.temp({nv, nv, nq}, false);
    o.vo = eng.temp({nv, no, nq}, false);
    eng.add(o.vv, reorder(Lv(Lvv, nv, nv), {1, 2, 0}), 1.0, 0.0, 0);
    eng.add(o.vo, reorder(Lv(Lov, no, nv), {2, 1, 0}), 1.0, 0.0, 0);
    return o;
  }

  void build_slab(const SlabOperands& L, int64_t e0, int64_t ce, const View& Vs, double* Wdst, const View& Bs,
                  double* Bpdst) {
    const int64_t Q = nq;
    {
      // the product lands in a GEMM-order temporary before it is permuted into
      // place: sub-slabs of e bound that temporary to kSlabDoubles
      const int64_t per_e = std::max<int64_t>(1, (int64_t)nv * nv * nv);
      const int64_t sub = std::max<int64_t>(1, std::min<int64_t>(ce, kSlabDoubles / per_e));
      // (ae|bf) = sum_Q L^Q_ae L^Q_bf
      for (int64_t k = 0; k < ce; k += sub) {
        const int64_t m = std::min<int64_t>(sub, ce - k);
        eng.contract("eaQ,fbQ->efab", block(L.vv, {e0 + k, 0, 0}, {m, nv, Q}), L.vv,
                     block(Vs, {k, 0, 0, 0}, {m, nv, nv, nv}), 1.0, 0);
      }
      // (me|bf) = sum_Q L^Q_me L^Q_bf
      const int64_t per_b = std::max<int64_t>(1, (int64_t)nv * no * nv);
      const int64_t sub_b = std::max<int64_t>(1, std::min<int64_t>(ce, kSlabDoubles / per_b));
      for (int64_t k = 0; k < ce; k += sub_b) {
        const int64_t m = std::min<int64_t>(sub_b, ce - k);
        eng.contract("emQ,fbQ->efmb", block(L.vo, {e0 + k, 0, 0}, {m, no, Q}), L.vv,
                     block(Bs, {k, 0, 0, 0}, {m, nv, no, nv}), 1.0, 0);
      }
    }
    SsOp w;
    w.mode = SsOp::kPackSlab;
    w.n1 = nv; w.n2 = nv; w.pair2 = 1; w.i0 = e0; w.ci = ce;
    w.x_re = Vs.re; w.y_re = Wdst;
    eng.ss(w);
    const size_t mk = arena.mark();
    View Xs = eng.temp({ce, nv, no, nv}, false);
    eng.add(Xs, Bs, 1.0, 0.0, 0);
    // (mf|be) for e in the slab: sum_Q L^Q_mf L^Q_be
    eng.contract("fmQ,ebQ->efmb", L.vo, block(L.vv, {e0, 0, 0}, {ce, nv, Q}), Xs, -1.0, 1);
    SsOp z;
    z.mode = SsOp::kPackSlab;
    z.n1 = nv; z.n2 = (int64_t)no * nv; z.pair2 = 0; z.i0 = e0; z.ci = ce;
    z.x_re = Xs.re; z.y_re = Bpdst;
    eng.ss(z);
    arena.release(mk);
  }

  void init(const double* eps, const double* chol) {
    setup_spaces();
    if (eps && core_orb >= 0) eps_core = eps[core_orb];
    eng.be = be;
    eng.scratch = &arena;
    eng.prec = RTEOM_FP64;   // integral blocks and Fock matrices: float64, once
    eng.dry = dry;
    const int64_t Q = nq;
    std::vector<int> ext(O);
    ext.insert(ext.end(), V.begin(), V.end());
    for (int s = 0; s < 2; ++s) {
      mo[s] = take(no);
      mv[s] = take(nv);
      fo[s] = take(no);
      fv[s] = take(nv);
      h2d(mo[s], mo_h[s].data(), no);
      h2d(mv[s], mv_h[s].data(), nv);
      f[s] = take((int64_t)nx * nx);
      h[s] = take((int64_t)nx * nx);
    }
    {
      const int64_t nt = 2 * npo() + 2 * npv();
      ptab = reinterpret_cast<int32_t*>(take((nt + 1) / 2));
      if (!dry) {
        std::vector<int32_t> t(nt);
        int64_t k = 0;
        for (int i = 0; i < no; ++i)
          for (int j = i + 1; j < no; ++j) { t[k] = i; t[npo() + k] = j; ++k; }
        k = 0;
        for (int a = 0; a < nv; ++a)
          for (int b = a + 1; b < nv; ++b) { t[2 * npo() + k] = a; t[2 * npo() + npv() + k] = b; ++k; }
        be->h2d(ptab, t.data(), nt * sizeof(int32_t));
      }
    }
    Loo = take(Q * no * no);
    Lov = take(Q * no * nv);
    Lvv = take(Q * nv * nv);
    Lvo = take(Q * nv * no);
    Jov = take((int64_t)no * nv * no * nv);
    Jx = take((int64_t)no * nv * no * nv);
    Jp = take(npv() * npo());
    if (plan.resident) {
      Vlad = take((int64_t)nv * nv * nv * nv);
      B1 = take((int64_t)nv * nv * no * nv);
      Wpp = take(npv() * npv());
      B1p = take(npv() * no * nv);
      if (opt.prec != RTEOM_FP64) {
        const int64_t v2 = (int64_t)nv * nv, pv = npv(), ov = (int64_t)no * nv;
        const std::pair<ConvSlot*, int64_t> slots[4] = {
            {&conv_v, conv_doubles(v2, v2)}, {&conv_w, conv_doubles(pv, pv)},
            {&conv_b1, conv_doubles(ov, v2)}, {&conv_b1p, conv_doubles(ov, pv)}};
        for (const auto& sl : slots) {
          *sl.first = ConvSlot();
          sl.first->doubles = sl.second;
          sl.first->p = take(sl.second);
        }
      }
    }
    const int64_t ns = lay.size();
    X = take(2 * ns);
    // one fixed pass per step forms the right-hand side in registers: no set for it
    RHS = opt.fp_fixed_iters == 1 ? nullptr : take(2 * ns);
    R = take(2 * ns);
    if (opt.fp_fixed_iters == 0) Tn = take(2 * ns);
    delta = take(1);
    dbad = take(1);
    epart = take(be ? be->energy_partials() : 4096);
    e_hist = take(2 * (opt.max_steps + 1));
    c_hist = take(2 * (opt.max_steps + 1));
    e_next = take(2);
    dstep = reinterpret_cast<int64_t*>(take(1));
    am = opt.fp_anderson;
    a_x.clear();
    a_f.clear();
    for (int j = 0; j < am; ++j) {
      a_x.push_back(take(2 * ns));
      a_f.push_back(take(2 * ns));
    }
    a_gram.assign(2 * (size_t)am * am, 0.0);
    a_dot = take(1);

    // Cholesky blocks in the extended ordering (host reorder, then copy)
    if (!dry) {
      std::vector<double> buf;
      auto put = [&](double* dst, int r0, int nr, int c0, int nc) {
        buf.resize((size_t)Q * nr * nc);
        for (int64_t q = 0; q < Q; ++q)
          for (int r = 0; r < nr; ++r) {
            const double* row = chol + ((size_t)q * n + ext[r0 + r]) * n;
            double* out = buf.data() + ((size_t)q * nr + r) * nc;
            for (int c = 0; c < nc; ++c) out[c] = row[ext[c0 + c]];
          }
        be->h2d(dst, buf.data(), buf.size() * sizeof(double));
      };
      put(Loo, 0, no, 0, no);
      put(Lov, 0, no, no, nv);
      put(Lvv, no, nv, no, nv);
      put(Lvo, no, nv, 0, no);
    }
    const size_t mk = arena.mark();
    // Fock of Phi per spin: f_pq = eps_p delta_pq - <pc||qc> (Sec. 2.1):
    // -(pq|cc) for both spins, +(pc|cq) for the spin of c.  The small vectors
    // L^Q_cc and L^Q_pc (p over the extended space) are gathered on the host.
    // (Without a core hole, core_orb < 0, f is the N-electron Fock matrix diag(eps).)
    View Lfull[2][2] = {{Lv(Loo, no, no), Lv(Lov, no, nv)}, {Lv(Lvo, nv, no), Lv(Lvv, nv, nv)}};
    const bool hole = core_orb >= 0;
    double* Lcc = take(Q);
    double* Lxc = take(Q * nx);
    double* dev_eps = take(nx);
    if (!dry) {
      std::vector<double> lcc(Q, 0.0), lxc((size_t)Q * nx, 0.0), epsx(nx);
      if (hole)
        for (int64_t q = 0; q < Q; ++q) {
          lcc[q] = chol[((size_t)q * n + core_orb) * n + core_orb];
          for (int p = 0; p < nx; ++p) lxc[(size_t)q * nx + p] = chol[((size_t)q * n + ext[p]) * n + core_orb];
        }
      for (int p = 0; p < nx; ++p) epsx[p] = eps[ext[p]];
      h2d(Lcc, lcc.data(), Q);
      h2d(Lxc, lxc.data(), Q * nx);
      h2d(dev_eps, epsx.data(), nx);
    }
    View Lxc_v = make_view(Lxc, nullptr, {Q, nx});
    for (int s = 0; s < 2; ++s) {
      View F = make_view(f[s], nullptr, {nx, nx});
      eng.add(F, F, 0.0, 0.0, 0);
      eng.add(diagonal(F, 0, 1), vec(dev_eps, nx), 1.0, 0.0, 0);
      for (int X1 = 0; X1 < 2; ++X1)
        for (int Y1 = 0; Y1 < 2; ++Y1) {
          const int64_t r0 = X1 ? no : 0, c0 = Y1 ? no : 0, nr = X1 ? nv : no, nc = Y1 ? nv : no;
          View blk = fview(f[s], r0, c0, nr, nc, false);
          if (!hole) continue;
          eng.contract("Qpq,Q->pq", Lfull[X1][Y1], vec(Lcc, Q), blk, -1.0, 1);
          if (s == core_spin)
            eng.contract("Qp,Qq->pq", block(Lxc_v, {0, r0}, {Q, nr}), block(Lxc_v, {0, c0}, {Q, nc}), blk, 1.0, 1);
        }
    }
    // h = f - J + K with J_pq = sum_Q L_pq j^Q, j^Q = sum_{s, k occ} L^Q_kk,
    // K^s_pq = sum_Q sum_{k occ in s} L_pk L_kq.
    View jq = make_view(take(Q), nullptr, {Q});
    for (int t = 0; t < 2; ++t)
      eng.contract("Qk,k->Q", diagonal(Lv(Loo, no, no), 1, 2), vec(mo[t], no), jq, 1.0, t);
    for (int s = 0; s < 2; ++s) {
      View H = make_view(h[s], nullptr, {nx, nx});
      eng.add(H, make_view(f[s], nullptr, {nx, nx}), 1.0, 0.0, 0);
      const double* sc_o[3] = {nullptr, nullptr, mo[s]};
      View Loo_m = make_view(take(Q * no * no), nullptr, {Q, no, no});
      View Lvo_m = make_view(take(Q * nv * no), nullptr, {Q, nv, no});
      eng.add(Loo_m, Lv(Loo, no, no), 1.0, 0.0, 0, sc_o);
      eng.add(Lvo_m, Lv(Lvo, nv, no), 1.0, 0.0, 0, sc_o);
      View Lpk[2] = {Loo_m, Lvo_m};
      for (int X1 = 0; X1 < 2; ++X1)
        for (int Y1 = 0; Y1 < 2; ++Y1) {
          View blk = fview(h[s], X1 ? no : 0, Y1 ? no : 0, X1 ? nv : no, Y1 ? nv : no, false);
          eng.contract("Qpq,Q->pq", Lfull[X1][Y1], jq, blk, -1.0, 1);
          eng.contract("Qpk,Qkq->pq", Lpk[X1], Lfull[0][Y1], blk, 1.0, 1);
        }
      // Fock diagonals for the diagonal map
      View Fo = block(diagonal(make_view(f[s], nullptr, {nx, nx}), 0, 1), {0}, {no});
      View Fv = block(diagonal(make_view(f[s], nullptr, {nx, nx}), 0, 1), {no}, {nv});
      eng.add(vec(fo[s], no), Fo, 1.0, 0.0, 0);
      eng.add(vec(fv[s], nv), Fv, 1.0, 0.0, 0);
    }
    arena.release(mk);
    // Resident integral blocks (spin free): (me|nf) and its pair form over (e<f), (m<n)
    eng.contract("Qme,Qnf->menf", Lv(Lov, no, nv), Lv(Lov, no, nv),
                 make_view(Jov, nullptr, {no, nv, no, nv}), 1.0, 0);
    // Jx[n][f][m][e] = (mf|ne) = Jov[m][f][n][e]
    eng.add(make_view(Jx, nullptr, {no, nv, no, nv}),
            reorder(make_view(Jov, nullptr, {no, nv, no, nv}), {2, 1, 0, 3}), 1.0, 0.0, 0);
    {
      const size_t mj = arena.mark();
      View t = eng.temp({nv, nv, no, no}, false);
      eng.add(t, reorder(make_view(Jov, nullptr, {no, nv, no, nv}), {1, 3, 0, 2}), 1.0, 0.0, 0);
      SsOp p;
      p.mode = SsOp::kPackSlab;
      p.n1 = nv; p.n2 = no; p.pair2 = 1; p.i0 = 0; p.ci = nv;
      p.x_re = t.re; p.y_re = Jp;
      eng.ss(p);   // Jp[e<f][m<n] = (me|nf) - (ne|mf)
      arena.release(mj);
    }
    if (plan.resident) {
      // built in slabs of e (GEMM-order temporaries bounded by kSlabDoubles)
      View Vv = make_view(Vlad, nullptr, {nv, nv, nv, nv});
      View Bv = make_view(B1, nullptr, {nv, nv, no, nv});
      const int64_t ce = std::max<int64_t>(1, std::min<int64_t>(nv, kSlabDoubles / std::max<int64_t>(1, (int64_t)nv * nv * nv)));
      const size_t ml = arena.mark();
      const SlabOperands L = slab_operands();
      for (int64_t e0 = 0; e0 < nv; e0 += ce) {
        const int64_t m = std::min<int64_t>(ce, nv - e0);
        build_slab(L, e0, m, block(Vv, {e0, 0, 0, 0}, {m, nv, nv, nv}), Wpp + pair_start(e0, nv) * npv(),
                   block(Bv, {e0, 0, 0, 0}, {m, nv, no, nv}), B1p + pair_start(e0, nv) * no * nv);
      }
      arena.release(ml);
    }
    // T(0) = 0, C(0) = 0
    if (!dry) {
      be->fill(X, 2 * ns, 0.0);
      be->fill(e_hist, 2, 0.0);
      be->fill(c_hist, 2, 0.0);
      be->fill(reinterpret_cast<double*>(dstep), 1, 0.0);   // all-zero bits: integer 0
      be->fill(dbad, 1, 0.0);
    }
    nsteps = 0;
    times.assign(1, 0.0);
    check();
  }

  // --------------------------------------------------------- residual
  // Integral products of the virtual slab e0 .. e0+ce-1: the particle-particle ladder
  // (alpha-beta in full storage, same-spin over pairs) and the Z intermediates.
  void slab_products(double* Xs, double* Rs, int64_t e0, int64_t ce, const View& Vs, double* Wsl, const View& Bs,
                     double* Bpsl, const View& Z3ab, const View& Zp, const View& Z2ab, bool first) {
    const int64_t r0 = pair_start(e0, nv), nr = pair_start(e0 + ce, nv) - r0;
    const int64_t nov = (int64_t)no * nv;
    const bool res = plan.resident;
    View Tab = block(tab3(Xs), {0, e0, 0}, {(int64_t)no * no, ce, nv});
    View Tp = block(tss2(Xs), {0, r0}, {2 * npo(), nr});
    eng.set_phase(kPhaseLadder);
    eng.contract("Pef,efab->Pab", Tab, Vs, tab3(Rs), 1.0, 1, res ? &conv_v : nullptr);
    if (nr > 0)
      eng.contract("Pr,rq->Pq", Tp, make_view(Wsl, nullptr, {nr, npv()}), tss2(Rs), 1.0, 1, res ? &conv_w : nullptr);
    eng.set_phase(kPhaseRing);
    // Z_ij,mb = sum_ef T_ijef (me|bf); same-spin: sum_{e<f} T_ijef [(me|bf) - (mf|be)]
    eng.contract("Pef,efmb->Pmb", Tab, Bs, Z3ab, 1.0, first ? 0 : 1, res ? &conv_b1 : nullptr);
    if (nr > 0)
      eng.contract("Pr,rc->Pc", Tp, make_view(Bpsl, nullptr, {nr, nov}), Zp, 1.0, first ? 0 : 1,
                   res ? &conv_b1p : nullptr);
    else if (first)
      eng.add(Zp, Zp, 0.0, 0.0, 0);
    // Z2_ij,an = sum_ef T_ijef (ae|nf), here over f in the slab: (me|bf) as [f][e][n][a]
    eng.contract("ijef,fena->ijan", block(tab(Xs), {0, 0, 0, e0}, {no, no, nv, ce}), Bs, Z2ab, 1.0, first ? 0 : 1);
    eng.set_phase(kPhaseGemm);
  }

  // Zero the amplitudes of spin-orbitals that do not exist.
  void mask_set(double* set) {
    for (int s = 0; s < 2; ++s) {
      const double* sc[2] = {mo[s], mv[s]};
      eng.scale(t1(set, s), sc);
      SsOp m = ss_op(SsOp::kMask, set, s);
      m.m1 = mo[s];
      m.m2 = mv[s];
      eng.ss(m);
    }
    const double* sc[4] = {mo[0], mo[1], mv[0], mv[1]};
    eng.scale(tab(set), sc);
  }

  // R <- <Phi_x| e^{-T} H_N e^{T} |Phi> for T = Xs (all five blocks, masked).
  void residual(double* Xs, double* Rs) {
    const int64_t Q = nq;
    const size_t mk = arena.mark();
    eng.prec = opt.prec;     // the residual's contractions in the requested precision
    eng.flops = eng.alg_flops = 0.0;
    for (int k = 0; k < kNumPhases; ++k) eng.phase_flops[k] = eng.alg_phase_flops[k] = 0.0;
    eng.set_phase(kPhaseGemm);
    t_res = std::chrono::steady_clock::now();
    fill(Rs, 2 * lay.size());        // every term below accumulates
    const int64_t nov = (int64_t)no * nv;
    const int64_t ci = std::max<int64_t>(1, std::min<int64_t>(plan.ci, no));
    const int64_t cj = std::max<int64_t>(1, std::min<int64_t>(plan.cj, no));
    View Lov_v = Lv(Lov, no, nv);
    View Jv = make_view(Jov, nullptr, {no, nv, no, nv});
    View Jxv = make_view(Jx, nullptr, {no, nv, no, nv});
    // intermediates that live through the whole evaluation
    View Ldoo[2], Ldvo[2], fd[2], D[2], Lbar[2], Fvv[2], Foo[2];
    for (int s = 0; s < 2; ++s) {
      Ldoo[s] = with_frac(eng.temp({Q, no, no}, true), {1, f_o[s], f_o[s]});
      Ldvo[s] = with_frac(eng.temp({Q, nv, no}, true), {1, f_v[s], f_o[s]});
      fd[s] = eng.temp({nx, nx}, true);
      D[s] = with_frac(eng.temp({Q, no, nv}, true), {1, f_o[s], f_v[s]});
      Lbar[s] = with_frac(eng.temp({Q, nv, no}, true), {1, f_v[s], f_o[s]});
      Fvv[s] = with_frac(eng.temp({nv, nv}, true), {f_v[s], f_v[s]});
      Foo[s] = with_frac(eng.temp({no, no}, true), {f_o[s], f_o[s]});
    }
    View jq = eng.temp({Q}, true);
    // the dressed virtual-virtual vectors are needed up to the ring intermediates only
    const size_t mk_vv = arena.mark();
    View Ldvv[2];
    for (int s = 0; s < 2; ++s) Ldvv[s] = with_frac(eng.temp({Q, nv, nv}, true), {1, f_v[s], f_v[s]});
    // dressed Cholesky vectors L~ = (1 - t) L (1 + t)
    for (int s = 0; s < 2; ++s) {
      View t = t1(Xs, s);
      eng.add(Ldoo[s], Lv(Loo, no, no), 1, 0, 0);
      eng.contract("Qmf,if->Qmi", Lov_v, t, Ldoo[s], 1.0, 1);
      eng.add(Ldvv[s], Lv(Lvv, nv, nv), 1, 0, 0);
      eng.contract("ma,Qme->Qae", t, Lov_v, Ldvv[s], -1.0, 1);
      eng.add(Ldvo[s], Lv(Lvo, nv, no), 1, 0, 0);
      eng.contract("Qaf,if->Qai", Lv(Lvv, nv, nv), t, Ldvo[s], 1.0, 1);
      eng.contract("ma,Qmi->Qai", t, Ldoo[s], Ldvo[s], -1.0, 1);
    }
    // dressed Fock of Phi: f~ = (1 - t) h (1 + t) + J~ - K~
    for (int t = 0; t < 2; ++t)
      eng.contract("Qk,k->Q", diagonal(Ldoo[t], 1, 2), vec(mo[t], no), jq, 1.0, t);
    for (int s = 0; s < 2; ++s) {
      const size_t mf = arena.mark();
      View t = t1(Xs, s);
      double* base = fd[s].re;
      View foo = fview(base, 0, 0, no, no, true), fov = fview(base, 0, no, no, nv, true);
      View fvo = fview(base, no, 0, nv, no, true), fvv = fview(base, no, no, nv, nv, true);
      View hoo = fview(h[s], 0, 0, no, no, false), hov = fview(h[s], 0, no, no, nv, false);
      View hvo = fview(h[s], no, 0, nv, no, false), hvv = fview(h[s], no, no, nv, nv, false);
      eng.add(foo, hoo, 1, 0, 0);
      eng.contract("mf,if->mi", hov, t, foo, 1.0, 1);
      eng.add(fov, hov, 1, 0, 0);
      eng.add(fvv, hvv, 1, 0, 0);
      eng.contract("ma,me->ae", t, hov, fvv, -1.0, 1);
      eng.add(fvo, hvo, 1, 0, 0);
      eng.contract("af,if->ai", hvv, t, fvo, 1.0, 1);
      eng.contract("ma,mi->ai", t, foo, fvo, -1.0, 1);   // uses the dressed h_oo only
      eng.contract("Qmi,Q->mi", Ldoo[s], jq, foo, 1.0, 1);
      eng.contract("Qme,Q->me", Lov_v, jq, fov, 1.0, 1);
      eng.contract("Qae,Q->ae", Ldvv[s], jq, fvv, 1.0, 1);
      eng.contract("Qai,Q->ai", Ldvo[s], jq, fvo, 1.0, 1);
      const double* sc[3] = {nullptr, nullptr, mo[s]};
      View Loo_m = eng.temp({Q, no, no}, true);
      View Lvo_m = eng.temp({Q, nv, no}, true);
      eng.add(Loo_m, Ldoo[s], 1, 0, 0, sc);
      eng.add(Lvo_m, Ldvo[s], 1, 0, 0, sc);
      eng.contract("Qmk,Qki->mi", Loo_m, Ldoo[s], foo, -1.0, 1);
      eng.contract("Qmk,Qke->me", Loo_m, Lov_v, fov, -1.0, 1);
      eng.contract("Qak,Qke->ae", Lvo_m, Lov_v, fvv, -1.0, 1);
      eng.contract("Qak,Qki->ai", Lvo_m, Ldoo[s], fvo, -1.0, 1);
      arena.release(mf);
    }
    // D^Q_ia = sum_{me} T_imae L^Q_me summed over the spin of (m, e), and the singles'
    // T2 terms, over blocks of rows i of the expanded same-spin amplitudes
    for (int s = 0; s < 2; ++s) {
      const int u = 1 - s;
      View r1 = t1(Rs, s);
      for (int64_t i0 = 0; i0 < no; i0 += ci) {
        const int64_t m = std::min<int64_t>(ci, no - i0);
        const size_t mr = arena.mark();
        // opposite-spin (m, e): the rows' block of the alpha-beta amplitudes (its (m, e)
        // sum is not one stride, so the engine stages the block, not the whole tensor)
        View tb = block(tsu(Xs, s), {i0, 0, 0, 0}, {m, no, nv, nv});
        View Db = block(D[s], {0, i0, 0}, {Q, m, nv}), r1b = block(r1, {i0, 0}, {m, nv});
        eng.contract("imae,Qme->Qia", tb, Lov_v, Db, 1.0, 0);
        eng.contract("me,imae->ia", fview(fd[u].re, 0, no, no, nv, true), tb, r1b, 1.0, 1);
        arena.release(mr);
        // same-spin (m, e)
        View xt = expand_rows(Xs, s, i0, m);
        eng.contract("imae,Qme->Qia", xt, Lov_v, Db, 1.0, 1);
        eng.contract("me,imae->ia", fview(fd[s].re, 0, no, no, nv, true), xt, r1b, 1.0, 1);
        arena.release(mr);
      }
      eng.add(Lbar[s], Ldvo[s], 1, 0, 0);
      eng.add(Lbar[s], reorder(D[s], {0, 2, 1}), 1, 0, 1);
      eng.add(Fvv[s], fview(fd[s].re, no, no, nv, nv, true), 1, 0, 0);
      eng.contract("Qmb,Qme->be", D[s], Lov_v, Fvv[s], -1.0, 1);
      eng.add(Foo[s], fview(fd[s].re, 0, 0, no, no, true), 1, 0, 0);
      eng.contract("Qme,Qje->mj", Lov_v, D[s], Foo[s], 1.0, 1);
      // remaining singles terms
      eng.add(r1, reorder(fview(fd[s].re, no, 0, nv, no, true), {1, 0}), 1, 0, 1);
      eng.contract("Qae,Qie->ia", Ldvv[s], D[s], r1, 1.0, 1);
      eng.contract("Qmi,Qma->ia", Ldoo[s], D[s], r1, -1.0, 1);
    }
    // Ring terms P(ij) P(ab) sum_me t_imae W_mbej through the intermediates
    // W[(m,e),(b,j)], built and used for a block of j at a time: exchange blocks
    // WX(s,u) (m, j in s; b, e in u) and the opposite-spin blocks V(s) (m, e in s;
    // j, b in u).
    eng.set_phase(kPhaseRing);
    for (int64_t j0 = 0; j0 < no; j0 += cj) {
      const int64_t n = std::min<int64_t>(cj, no - j0);
      const size_t mw = arena.mark();
      View WX[2][2], Vx[2];
      for (int s = 0; s < 2; ++s)
        for (int u = 0; u < 2; ++u) {
          WX[s][u] = with_frac(eng.temp({no, nv, nv, n}, true), {f_o[s], f_v[u], f_v[u], f_o[s]});
          eng.contract("Qmj,Qbe->mbej", block(Ldoo[s], {0, 0, j0}, {Q, no, n}), Ldvv[u], WX[s][u], -1.0, 0);
          const size_t mr = arena.mark();
          View tj = s == u ? expand_rows(Xs, s, j0, n) : block(tsu(Xs, s), {j0, 0, 0, 0}, {n, no, nv, nv});
          eng.contract("jnfb,nfme->mbej", tj, Jxv, WX[s][u], 0.5, 1);
          arena.release(mr);
        }
      for (int s = 0; s < 2; ++s) {
        const int u = 1 - s;
        Vx[s] = with_frac(eng.temp({no, nv, nv, n}, true), {f_o[s], f_v[u], f_v[s], f_o[u]});
        eng.contract("jnbf,nfme->mbej", block(tsu(Xs, u), {j0, 0, 0, 0}, {n, no, nv, nv}), Jxv, Vx[s], -0.5, 0);
      }
      // same-spin residuals: x[i][j] over blocks of rows i, antisymmetrised into pairs
      for (int s = 0; s < 2; ++s) {
        const int u = 1 - s;
        for (int64_t i0 = 0; i0 < no; i0 += ci) {
          const int64_t m = std::min<int64_t>(ci, no - i0);
          const size_t mr = arena.mark();
          View x = sstemp({m, n, nv, nv}, s);
          View xt = expand_rows(Xs, s, i0, m);
          eng.contract("imae,mbej->ijab", xt, WX[s][s], x, 1.0, 0);
          eng.contract("imae,mbej->ijab", block(tsu(Xs, s), {i0, 0, 0, 0}, {m, no, nv, nv}), Vx[u], x, 1.0, 1);
          accum(Rs, s, x, i0, j0, 1.0, 1, 1);
          arena.release(mr);
        }
      }
      // alpha-beta residual (full storage): blocks of the residual's first two indices,
      // one of them the intermediate's last index j (the W block), the other a block of
      // the amplitudes' free occupied index
      View Rab = tab(Rs), Tab = tab(Xs);
      for (int64_t i0 = 0; i0 < no; i0 += ci) {
        const int64_t m = std::min<int64_t>(ci, no - i0);
        View Ti = block(Tab, {i0, 0, 0, 0}, {m, no, nv, nv});   // rows i of t_{i alpha, m beta}
        View Tj = block(Tab, {0, i0, 0, 0}, {no, m, nv, nv});   // columns j of t_{m alpha, j beta}
        View Rij = block(Rab, {i0, j0, 0, 0}, {m, n, nv, nv});  // i in the amplitude block, j in W's
        View Rji = block(Rab, {j0, i0, 0, 0}, {n, m, nv, nv});  // i in W's block, j in the amplitude block
        eng.contract("imae,mbej->ijab", Ti, WX[1][1], Rij, 1.0, 1);
        eng.contract("mjae,mbei->ijab", Tj, WX[0][1], Rji, 1.0, 1);
        eng.contract("imeb,maej->ijab", Ti, WX[1][0], Rij, 1.0, 1);
        eng.contract("mjeb,maei->ijab", Tj, WX[0][0], Rji, 1.0, 1);
        const size_t mr = arena.mark();
        View xa = expand_rows(Xs, 0, i0, m);
        eng.contract("imae,mbej->ijab", xa, Vx[0], Rij, 1.0, 1);
        arena.release(mr);
        View xb = expand_rows(Xs, 1, i0, m);
        eng.contract("jmbe,maei->ijab", xb, Vx[1], Rji, 1.0, 1);
        arena.release(mr);
      }
      arena.release(mw);
      if (cj < no) progress("ring block", std::min<int64_t>(j0 + cj, no), no);
    }
    eng.set_phase(kPhaseGemm);
    arena.release(mk_vv);
    // Z intermediates (from the integral slabs on)
    View Z3ab = with_frac(eng.temp({(int64_t)no * no, no, nv}, true), {f_o[0] * f_o[1], f_o[0], f_v[1]});
    View Zp = eng.temp({2 * npo(), nov}, true);
    View Z2ab = with_frac(eng.temp({no, no, nv, no}, true), {f_o[0], f_o[1], f_v[0], f_o[1]});
    // Particle-particle ladder and Z intermediates over virtual slabs of e: the resident
    // blocks at once, or each slab rebuilt from the Cholesky vectors
    if (plan.resident) {
      slab_products(Xs, Rs, 0, nv, make_view(Vlad, nullptr, {nv, nv, nv, nv}), Wpp,
                    make_view(B1, nullptr, {nv, nv, no, nv}), B1p, Z3ab, Zp, Z2ab, true);
    } else {
      const int64_t es = std::max<int64_t>(1, std::min<int64_t>(plan.es, nv));
      eng.set_phase(kPhaseBuild);
      const SlabOperands L = slab_operands();
      eng.set_phase(kPhaseGemm);
      for (int64_t e0 = 0; e0 < nv; e0 += es) {
        const int64_t ce = std::min<int64_t>(es, nv - e0);
        const int64_t nr = pair_start(e0 + ce, nv) - pair_start(e0, nv);
        const size_t ms = arena.mark();
        double* Wsl = take(std::max<int64_t>(1, nr * npv()));
        double* Bpsl = take(std::max<int64_t>(1, nr * nov));
        View Vs = eng.temp({ce, nv, nv, nv}, false);
        View Bs = eng.temp({ce, nv, no, nv}, false);
        eng.set_phase(kPhaseBuild);
        build_slab(L, e0, ce, Vs, Wsl, Bs, Bpsl);
        eng.set_phase(kPhaseGemm);
        slab_products(Xs, Rs, e0, ce, Vs, Wsl, Bs, Bpsl, Z3ab, Zp, Z2ab, e0 == 0);
        arena.release(ms);
        if ((e0 / es) % 8 == 7 || e0 + ce >= nv) progress("integral slab", e0 + ce, nv);
      }
    }
    // same-spin doubles: the terms in full storage over blocks of rows, the hole
    // ladders and the Z term in pair storage
    for (int s = 0; s < 2; ++s) {
      View t = t1(Xs, s);
      for (int64_t i0 = 0; i0 < no; i0 += ci) {
        const int64_t m = std::min<int64_t>(ci, no - i0);
        const size_t mr = arena.mark();
        View x = sstemp({m, no, nv, nv}, s);
        // dressed <ab||ij> plus Coulomb ring: Lbar_ai Lbar_bj - Lbar_aj Lbar_bi
        eng.contract("Qai,Qbj->ijab", block(Lbar[s], {0, 0, i0}, {Q, nv, m}), Lbar[s], x, 1.0, 0);
        accum(Rs, s, x, i0, 0, 1.0, 1, 0);
        View xt = expand_rows(Xs, s, i0, m);
        // P(ab) sum_e t_ijae F_be
        eng.contract("ijae,be->ijab", xt, Fvv[s], x, 1.0, 0);
        accum(Rs, s, x, i0, 0, 1.0, 0, 1);
        // -P(ij) sum_m t_imab F_mj
        eng.contract("imab,mj->ijab", xt, Foo[s], x, 1.0, 0);
        accum(Rs, s, x, i0, 0, -1.0, 1, 0);
        arena.release(mr);
      }
      const size_t mh = arena.mark();
      View Tp = tss(Xs, s), Rp = tss(Rs, s);
      // hole ladder: 1/2 sum_mn t_mnab gA_mnij = sum_{m<n} gA[m<n][i<j] t[m<n][a<b], with
      // gA_mnij = g_mnij - g_mnji, g = sum_Q L~_mi L~_nj (T1-T1 piece of the ladder)
      View g = eng.temp({no, no, no, no}, true);
      eng.contract("Qmi,Qnj->mnij", Ldoo[s], Ldoo[s], g, 1.0, 0);
      View gA = with_frac(eng.temp({npo(), npo()}, true), {f_po[s], f_po[s]});
      {
        SsOp p;
        p.mode = SsOp::kPackSlab;
        p.n1 = no; p.n2 = no; p.pair2 = 1; p.i0 = 0; p.ci = no;
        p.x_re = g.re; p.x_im = g.im; p.y_re = gA.re; p.y_im = gA.im;
        eng.ss(p);
      }
      eng.contract("rp,rq->pq", gA, Tp, Rp, 1.0, 1);
      // 1/2 sum_mn tau_mnab Xo_ijmn over pairs, Xo_ijmn = sum_ef t_ijef (me|nf)
      View Xo = with_frac(eng.temp({npo(), npo()}, true), {f_po[s], f_po[s]});
      eng.contract("pr,rm->pm", Tp, make_view(Jp, nullptr, {npv(), npo()}), Xo, 1.0, 0);
      View tau = with_frac(eng.temp({npo(), npv()}, true), {f_po[s], f_pv[s]});
      eng.add(tau, Tp, 1, 0, 0);
      {
        SsOp p;
        p.mode = SsOp::kT1T1;
        p.n1 = no; p.n2 = nv; p.beta = 1; p.alpha = 1.0;
        p.y_re = tau.re; p.y_im = tau.im; p.u_re = t.re; p.u_im = t.im;
        p.pt = tables();
        eng.ss(p);
      }
      eng.contract("pm,mq->pq", Xo, tau, Rp, 1.0, 1);
      arena.release(mh);
      // Z: -P(ab) sum_m t_ma Z_ij,mb over pairs i<j (blocks of pair rows)
      const int64_t cp = std::max<int64_t>(1, std::min<int64_t>(npo(), kPairRowDoubles / std::max<int64_t>(1, 2 * (int64_t)nv * nv)));
      for (int64_t p0 = 0; p0 < npo(); p0 += cp) {
        const int64_t m = std::min<int64_t>(cp, npo() - p0);
        const size_t mr = arena.mark();
        View y = with_frac(eng.temp({m, nv, nv}, true), {f_po[s], f_v[s], f_v[s]});
        View Zs = with_frac(make_view(Zp.re + (s * npo() + p0) * nov, Zp.im + (s * npo() + p0) * nov, {m, no, nv}),
                            {f_po[s], f_o[s], f_v[s]});
        eng.contract("ma,Pmb->Pab", t, Zs, y, -1.0, 0);
        SsOp a = ss_op(SsOp::kAccumRows, Rs, s);
        a.i0 = p0; a.ci = m; a.anti2 = 1;
        a.x_re = y.re; a.x_im = y.im;
        eng.ss(a);
        arena.release(mr);
      }
    }
    // alpha-beta doubles (full storage, accumulated in place)
    {
      View Rv = tab(Rs), T = tab(Xs);
      View ta = t1(Xs, 0), tb = t1(Xs, 1);
      // Products whose operand or result the engine stages (no single stride over a
      // summed or an output index pair) run over blocks of one occupied index, so that
      // the staged copies are blocks, not whole o^2 v^2 tensors
      for (int64_t i0 = 0; i0 < no; i0 += ci) {
        const int64_t m = std::min<int64_t>(ci, no - i0);
        eng.contract("Qai,Qbj->ijab", block(Lbar[0], {0, 0, i0}, {Q, nv, m}), Lbar[1],
                     block(Rv, {i0, 0, 0, 0}, {m, no, nv, nv}), 1.0, 1);
      }
      eng.contract("ijae,be->ijab", T, Fvv[1], Rv, 1.0, 1);
      eng.contract("ae,ijeb->ijab", Fvv[0], T, Rv, 1.0, 1);
      eng.contract("imab,mj->ijab", T, Foo[1], Rv, -1.0, 1);
      for (int64_t j0 = 0; j0 < no; j0 += cj) {
        const int64_t m = std::min<int64_t>(cj, no - j0);
        eng.contract("mi,mjab->ijab", Foo[0], block(T, {0, j0, 0, 0}, {no, m, nv, nv}),
                     block(Rv, {0, j0, 0, 0}, {no, m, nv, nv}), -1.0, 1);
      }
      const size_t ma = arena.mark();
      View g = with_frac(eng.temp({no, no, no, no}, true), {f_o[0], f_o[1], f_o[0], f_o[1]});
      View Xo = with_frac(eng.temp({no, no, no, no}, true), {f_o[0], f_o[1], f_o[0], f_o[1]});
      View Y = with_frac(eng.temp({no, no, no, nv}, true), {f_o[0], f_o[1], f_o[0], f_v[1]});
      eng.contract("Qmi,Qnj->mnij", Ldoo[0], Ldoo[1], g, 1.0, 0);
      for (int64_t m0 = 0; m0 < no; m0 += ci) {
        const int64_t m = std::min<int64_t>(ci, no - m0);
        eng.contract("ijef,menf->ijmn", T, block(Jv, {m0, 0, 0, 0}, {m, nv, no, nv}),
                     block(Xo, {0, 0, m0, 0}, {no, no, m, no}), 1.0, 0);
      }
      eng.contract("mnab,mnij->ijab", T, g, Rv, 1.0, 1);
      // sum_mn tau_mnab Xo_ijmn with tau = t2 + t_ma t_nb
      eng.contract("mnab,ijmn->ijab", T, Xo, Rv, 1.0, 1);
      eng.contract("ijmn,nb->ijmb", Xo, tb, Y, 1.0, 0);
      eng.contract("ma,ijmb->ijab", ta, Y, Rv, 1.0, 1);
      eng.contract("ma,ijmb->ijab", ta, make_view(Z3ab.re, Z3ab.im, {no, no, no, nv}), Rv, -1.0, 1);
      eng.contract("nb,ijan->ijab", tb, Z2ab, Rv, -1.0, 1);
      arena.release(ma);
    }
    mask_set(Rs);
    res_flops = eng.flops;
    res_alg_flops = eng.alg_flops;
    for (int k = 0; k < kNumPhases; ++k) {
      res_phase_flops[k] = eng.phase_flops[k];
      res_alg_phase_flops[k] = eng.alg_phase_flops[k];
    }
    eng.prec = RTEOM_FP64;
    arena.release(mk);
  }

  // ------------------------------------------------------------- energy
  void energy(double* Xs, double* e_out) {
    EnergyOp op;
    op.lay = lay;
    op.x_re = Xs;
    op.x_im = Xs + lay.size();
    op.jov = Jov;
    op.fov[0] = f[0] + no;
    op.fov[1] = f[1] + no;
    op.fov_ld = nx;
    op.include_ft1 = opt.dC_include_fT1;
    op.e_out = e_out;
    op.partial = epart;
    if (!dry) be->energy(op);
  }

  UpdateOp update_op(bool start) {
    UpdateOp u;
    u.lay = lay;
    u.pt = tables();
    u.x_re = X;
    u.x_im = X + lay.size();
    u.r_re = R;
    u.r_im = R + lay.size();
    u.rhs_re = RHS;
    u.rhs_im = RHS ? RHS + lay.size() : nullptr;
    u.mode = opt.fp_map;
    u.start = start ? 1 : 0;
    for (int s = 0; s < 2; ++s) {
      u.sv.mo[s] = mo[s];
      u.sv.mv[s] = mv[s];
      u.sv.fo[s] = fo[s];
      u.sv.fv[s] = fv[s];
    }
    u.delta = delta;
    return u;
  }

  // --------------------------------------------------------------- step
  // One step of Eq. trapzrule: R_n = R(T_n); rhs = T_n + (i dt/2) R_n;
  // T^(1) = rhs + (i dt/2) R_n; T^(k+1) = rhs + (i dt/2) R(T^(k)).
  int step(double dt) {
    if (nsteps >= opt.max_steps) throw Error(RTEOM_ERR_STATE, "C(t) history is full (max_steps)");
    const int passes = enqueue_step(dt);
    ++nsteps;
    times.push_back(times.back() + dt);
    return passes;
  }

  // After the stream has drained: did any step of the call append a non-finite E or C?
  void check_finite() {
    if (dry) return;
    double b = 0.0;
    be->d2h(&b, dbad, sizeof(double));
    if (b != 0.0)
      throw Error(RTEOM_ERR_NONFINITE, "non-finite amplitudes: E(T) or C(t) of step " + std::to_string(nsteps) +
                                           " or earlier is NaN or infinite");
  }

  // Fixed-pass steps may be captured once into a graph and replayed: every
  // argument of a step is either constant or read from device memory.
  bool graph_mode() const { return opt.graph != 0 && opt.fp_fixed_iters > 0; }
  void* graph_for(double dt) {
    if (step_graph && graph_dt == dt) return step_graph;
    if (step_graph) {
      be->destroy_graph(step_graph);
      step_graph = nullptr;
    }
    if (!be->begin_capture()) return nullptr;
    enqueue_step(dt);
    step_graph = be->end_capture();
    graph_dt = dt;
    check();
    return step_graph;
  }
  int step_graphed(double dt) {
    if (nsteps >= opt.max_steps) throw Error(RTEOM_ERR_STATE, "C(t) history is full (max_steps)");
    void* g = graph_for(dt);
    if (!g) return step(dt);
    be->launch_graph(g);
    ++nsteps;
    times.push_back(times.back() + dt);
    return opt.fp_fixed_iters;
  }

  // ---- Anderson acceleration (type II, Pulay/DIIS form) of a fixed point x = G(x):
  // with f_j = G(x_j) - x_j over the last c <= am iterates, the next iterate is
  // sum_j a_j G(x_j) with the complex a_j (sum 1) that minimise |sum_j a_j f_j|_2.
  // Complex weights: the error modes of the time-step map rotate in the complex
  // plane (the i dt/2 factor), which real weights cannot cancel.
  View flat(double* set) const { return make_view(set, nullptr, {2 * lay.size()}); }
  View cplx(double* set) const { return make_view(set, set + lay.size(), {lay.size()}); }
  void anderson_reset() { a_count = 0; a_head = 0; }
  // before G is applied to X: keep x
  void anderson_keep_x() { be->d2d(a_x[a_head], X, sizeof(double) * 2 * lay.size()); }
  double dot(const double* a, const double* b, int64_t n) {
    double d = 0.0;
    be->dot(a, b, n, epart, a_dot);
    be->d2h(&d, a_dot, sizeof(double));
    return d;
  }
  // after X = G(x): record f = G(x) - x and replace X by the mixed iterate
  void anderson_mix() {
    typedef std::complex<double> cd;
    const int h = a_head;
    const int64_t ns = lay.size();
    eng.set_phase(kPhaseMove);
    eng.add(flat(a_f[h]), flat(X), 1.0, 0.0, 0);
    eng.add(flat(a_f[h]), flat(a_x[h]), -1.0, 0.0, 1);
    a_count = std::min(a_count + 1, am);
    std::vector<int> slots;   // oldest first
    for (int k = a_count - 1; k >= 0; --k) slots.push_back((h - k + am) % am);
    for (int j : slots) {
      // <f_h, f_j> = sum conj(f_h) f_j
      const double re = dot(a_f[h], a_f[j], 2 * ns);
      const double im = j == h ? 0.0 : dot(a_f[h], a_f[j] + ns, ns) - dot(a_f[h] + ns, a_f[j], ns);
      a_gram[2 * ((size_t)h * am + j)] = re;
      a_gram[2 * ((size_t)h * am + j) + 1] = im;
      a_gram[2 * ((size_t)j * am + h)] = re;
      a_gram[2 * ((size_t)j * am + h) + 1] = -im;
    }
    a_head = (h + 1) % am;
    const int c = (int)slots.size();
    if (c < 2) return;   // X = G(x) as it stands
    // [B 1; 1^T 0] [a; l] = [0; 1], B_ij = <f_i, f_j>, by elimination with pivoting
    const int n1 = c + 1;
    std::vector<cd> A((size_t)n1 * n1, cd(0.0)), rhs(n1, cd(0.0));
    double scale = 0.0;
    for (int i = 0; i < c; ++i) scale = std::max(scale, a_gram[2 * ((size_t)slots[i] * am + slots[i])]);
    if (!(scale > 0.0)) return;
    for (int i = 0; i < c; ++i) {
      for (int j = 0; j < c; ++j) {
        const size_t g = 2 * ((size_t)slots[i] * am + slots[j]);
        A[(size_t)i * n1 + j] = cd(a_gram[g], a_gram[g + 1]) / scale;
      }
      A[(size_t)i * n1 + i] *= 1.0 + 1e-12;
      A[(size_t)i * n1 + c] = A[(size_t)c * n1 + i] = cd(1.0);
    }
    rhs[c] = cd(1.0);
    for (int col = 0; col < n1; ++col) {
      int piv = col;
      for (int r = col + 1; r < n1; ++r)
        if (std::abs(A[(size_t)r * n1 + col]) > std::abs(A[(size_t)piv * n1 + col])) piv = r;
      if (std::abs(A[(size_t)piv * n1 + col]) < 1e-300) return;   // degenerate: keep G(x)
      for (int k = 0; k < n1; ++k) std::swap(A[(size_t)col * n1 + k], A[(size_t)piv * n1 + k]);
      std::swap(rhs[col], rhs[piv]);
      for (int r = col + 1; r < n1; ++r) {
        const cd fct = A[(size_t)r * n1 + col] / A[(size_t)col * n1 + col];
        for (int k = col; k < n1; ++k) A[(size_t)r * n1 + k] -= fct * A[(size_t)col * n1 + k];
        rhs[r] -= fct * rhs[col];
      }
    }
    std::vector<cd> a(n1, cd(0.0));
    for (int r = n1 - 1; r >= 0; --r) {
      cd v = rhs[r];
      for (int k = r + 1; k < n1; ++k) v -= A[(size_t)r * n1 + k] * a[k];
      a[r] = v / A[(size_t)r * n1 + r];
    }
    for (int i = 0; i < c; ++i)
      if (!std::isfinite(a[i].real()) || !std::isfinite(a[i].imag())) return;
    // X = sum_j a_j (x_j + f_j), complex a_j on planar complex sets
    for (int i = 0; i < c; ++i) {
      eng.add(cplx(X), cplx(a_x[slots[i]]), a[i].real(), a[i].imag(), i == 0 ? 0 : 1);
      eng.add(cplx(X), cplx(a_f[slots[i]]), a[i].real(), a[i].imag(), 1);
    }
  }

  // Ground-state CCSD (R(T) = 0) by Jacobi iteration from T = 0; e_out = E^corr.
  int ground_state(double tol, int max_iter, double* e_out) {
    be->fill(X, 2 * lay.size(), 0.0);
    UpdateOp u = update_op(false);
    u.mode = 2;
    anderson_reset();
    for (int it = 1; it <= max_iter; ++it) {
      residual(X, R);
      if (am > 0) anderson_keep_x();
      be->set_phase(kPhaseUpdate);
      be->fill(delta, 1, 0.0);
      be->update(u);
      double d = 0.0;
      be->d2h(&d, delta, sizeof(double));
      if (!std::isfinite(d)) throw Error(RTEOM_ERR_NONFINITE, "non-finite amplitudes in the ground-state iteration");
      if (d < tol) {
        be->set_phase(kPhaseEnergy);
        energy(X, e_next);
        be->d2h(e_out, e_next, 2 * sizeof(double));
        return it;
      }
      if (am > 0) anderson_mix();
    }
    throw Error(RTEOM_ERR_NOCONV, "ground-state CCSD not converged in " + std::to_string(max_iter) + " iterations");
  }

  // A tolerance-driven step that fails puts T_n back: the step is not committed.
  [[noreturn]] void fail_step(int code, const std::string& m) {
    be->d2d(X, Tn, sizeof(double) * 2 * lay.size());
    be->sync();
    restored = true;
    throw Error(code, m);
  }

  int enqueue_step(double dt) {
    UpdateOp u0 = update_op(true);
    u0.h = 0.5 * dt;
    const bool accel = am > 0 && opt.fp_fixed_iters == 0;   // tolerance-driven passes only
    restored = false;
    if (opt.fp_fixed_iters == 0) be->d2d(Tn, X, sizeof(double) * 2 * lay.size());
    if (accel) anderson_reset();
    residual(X, R);
    if (accel) anderson_keep_x();
    be->set_phase(kPhaseUpdate);
    be->fill(delta, 1, 0.0);
    be->update(u0);
    int passes = 1;
    UpdateOp u = update_op(false);
    u.h = 0.5 * dt;
    if (opt.fp_fixed_iters > 0) {
      while (passes < opt.fp_fixed_iters) {
        residual(X, R);
        be->set_phase(kPhaseUpdate);
        be->fill(delta, 1, 0.0);
        be->update(u);
        ++passes;
      }
    } else {
      double d = 0.0;
      be->d2h(&d, delta, sizeof(double));
      while (!(d < opt.fp_tol)) {
        if (!std::isfinite(d)) fail_step(RTEOM_ERR_NONFINITE, "non-finite amplitudes in the fixed point");
        if (passes >= opt.fp_max_iter)
          fail_step(RTEOM_ERR_NOCONV, "fixed point not converged after " + std::to_string(passes) +
                                          " passes (last change " + std::to_string(d) + ")");
        if (accel) anderson_mix();
        residual(X, R);
        if (accel) anderson_keep_x();
        be->set_phase(kPhaseUpdate);
        be->fill(delta, 1, 0.0);
        be->update(u);
        ++passes;
        be->d2h(&d, delta, sizeof(double));
      }
    }
    be->set_phase(kPhaseEnergy);
    energy(X, e_next);
    be->cumulant_append(c_hist, e_hist, e_next, dstep, 0.5 * dt, dbad);
    return passes;
  }
};

}  // namespace rteom

using rteom::Context;
using rteom::Error;

struct rteom_ctx {
  Context c;
};

namespace {
std::string g_last_error;

void fail(rteom_ctx* ctx, const std::string& m) {
  if (ctx) ctx->c.err = m; else g_last_error = m;
}

template <class F>
rteom_status guarded(rteom_ctx* ctx, F&& fn) {
  try {
    fn();
    if (ctx && !ctx->c.dry) {
      std::string m;
      if (!ctx->c.be->ok(&m)) {
        fail(ctx, m);
        return RTEOM_ERR_HIP;
      }
    }
    return RTEOM_OK;
  } catch (const Error& e) {
    fail(ctx, e.what());
    return static_cast<rteom_status>(e.code);
  } catch (const std::bad_alloc&) {
    fail(ctx, "host allocation failed");
    return RTEOM_ERR_OOM;
  } catch (const std::exception& e) {
    fail(ctx, e.what());
    return RTEOM_ERR_HIP;
  }
}

bool valid_options(const rteom_options* o, std::string* m) {
  if (o->struct_size != sizeof(rteom_options)) { *m = "rteom_options.struct_size mismatch"; return false; }
  if (o->prec < 0 || o->prec > 3) { *m = "unknown precision"; return false; }
  if (o->fp_map < 0 || o->fp_map > 1) { *m = "unknown fixed-point map"; return false; }
  if (o->fp_fixed_iters < 0 || o->fp_max_iter < 1) { *m = "bad pass counts"; return false; }
  if (!(o->fp_tol > 0.0)) { *m = "fp_tol must be positive"; return false; }
  if (o->max_steps < 1) { *m = "max_steps must be >= 1"; return false; }
  if (o->tune < 0 || o->tune > 1) { *m = "tune must be 0 or 1"; return false; }
  if (o->fp_anderson < 0 || o->fp_anderson > 8) { *m = "fp_anderson must be in 0..8"; return false; }
  if (o->plan_slab < 0 || o->plan_block < 0) { *m = "plan_slab and plan_block must be >= 0"; return false; }
  return true;
}

// Memory limit of the plan: the option (0 = the default), and no more than a caller's workspace.
size_t plan_limit(const rteom_options& o) {
  size_t lim = o.mem_limit ? o.mem_limit : rteom::kDefaultMemLimit;
  if (o.workspace) lim = std::min(lim, o.workspace_bytes);
  return lim;
}

rteom_status check_sizes(int32_t n_orb, int32_t n_occ_a, int32_t n_occ_b, int32_t n_chol,
                         int32_t core_orb, int32_t core_spin, std::string* m) {
  if (n_orb < 2 || n_chol < 1) { *m = "n_orb >= 2 and n_chol >= 1 required"; return RTEOM_ERR_ARG; }
  if (n_occ_a < 0 || n_occ_b < 0 || n_occ_a > n_orb || n_occ_b > n_orb) { *m = "bad occupation numbers"; return RTEOM_ERR_ARG; }
  if (core_orb != -1) {   // -1: the N-electron determinant itself (no core hole)
    if (core_spin != 0 && core_spin != 1) { *m = "core_spin must be 0 (alpha) or 1 (beta)"; return RTEOM_ERR_ARG; }
    const int nocc = core_spin == 0 ? n_occ_a : n_occ_b;
    if (core_orb < 0 || core_orb >= nocc) { *m = "core orbital is not occupied in that spin"; return RTEOM_ERR_ARG; }
  }
  if (n_occ_a + n_occ_b < 2) { *m = "need at least two electrons"; return RTEOM_ERR_ARG; }
  return RTEOM_OK;
}
}  // namespace

extern "C" {

void rteom_default_options(rteom_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(rteom_options);
  o->prec = RTEOM_FP64;
  o->fp_map = 0;
  o->fp_fixed_iters = 0;
  o->fp_max_iter = 50;
  o->fp_tol = 1e-10;
  o->dC_include_fT1 = 1;
  o->max_steps = 100000;
  o->tune = 1;
}

// What one dry run of init + one residual (no device work) gives.
struct PlanResult {
  rteom::Plan plan;
  size_t bytes = 0;
  double flops = 0.0, alg_flops = 0.0;
  double phase_flops[rteom::kNumPhases] = {0}, alg_phase_flops[rteom::kNumPhases] = {0};
};

static rteom_status dry_run(int32_t n_orb, int32_t n_occ_a, int32_t n_occ_b, int32_t n_chol, int32_t core_orb,
                            int32_t core_spin, const rteom_options& o, const rteom::Plan& plan, PlanResult* r) {
  std::unique_ptr<rteom_ctx> ctx(new rteom_ctx());
  Context& c = ctx->c;
  c.dry = true;
  c.opt = o;
  c.plan = plan;
  c.n = n_orb; c.nq = n_chol; c.na = n_occ_a; c.nb = n_occ_b; c.core_orb = core_orb; c.core_spin = core_spin;
  c.arena.init(nullptr, ~static_cast<size_t>(0) >> 2);
  const rteom_status st = guarded(ctx.get(), [&] {
    c.init(nullptr, nullptr);
    c.residual(c.X, c.R);
  });
  if (st != RTEOM_OK) { g_last_error = c.err; return st; }
  r->plan = plan;
  r->bytes = c.arena.peak() + (1 << 20);
  r->flops = c.res_flops;
  r->alg_flops = c.res_alg_flops;
  for (int k = 0; k < rteom::kNumPhases; ++k) {
    r->phase_flops[k] = c.res_phase_flops[k];
    r->alg_phase_flops[k] = c.res_alg_phase_flops[k];
  }
  return RTEOM_OK;
}

// The plan of the largest blocks whose workspace fits the memory limit: the integral
// blocks resident and no blocking if possible, then smaller ring and row blocks, then
// integral slabs rebuilt per residual (largest slab first).
static rteom_status choose_plan(int32_t n_orb, int32_t n_occ_a, int32_t n_occ_b, int32_t n_chol, int32_t core_orb,
                                int32_t core_spin, const rteom_options& o, PlanResult* out) {
  const size_t lim = plan_limit(o);
  const int64_t all = int64_t(1) << 30;
  std::vector<rteom::Plan> cands;
  if (o.plan_slab > 0 || o.plan_block > 0) {
    const int64_t c = o.plan_block > 0 ? o.plan_block : all;
    cands.push_back({o.plan_slab == 0, (int64_t)o.plan_slab, c, c});
  } else {
    for (int64_t c : {all, int64_t(32), int64_t(16), int64_t(8), int64_t(4), int64_t(2), int64_t(1)})
      cands.push_back({true, 0, c, c});
    const int64_t slab[][2] = {{16, 16}, {8, 8}, {16, 8}, {8, 4}, {4, 4}, {2, 2}, {1, 1}};
    for (const auto& x : slab) cands.push_back({false, x[0], x[1], x[1]});
  }
  size_t smallest = ~size_t(0);
  for (const rteom::Plan& p : cands) {
    PlanResult r;
    const rteom_status st = dry_run(n_orb, n_occ_a, n_occ_b, n_chol, core_orb, core_spin, o, p, &r);
    if (st != RTEOM_OK) return st;
    if (r.bytes <= lim) {
      *out = r;
      return RTEOM_OK;
    }
    smallest = std::min(smallest, r.bytes);
  }
  g_last_error = "no plan fits the memory limit of " + std::to_string(lim) + " bytes (smallest needs " +
                 std::to_string(smallest) + ")";
  return RTEOM_ERR_OOM;
}

rteom_status rteom_workspace_query(int32_t n_orb, int32_t n_occ_a, int32_t n_occ_b, int32_t n_chol,
                                   int32_t core_orb, int32_t core_spin, const rteom_options* opt,
                                   size_t* bytes) {
  std::string m;
  if (!bytes) { g_last_error = "bytes is NULL"; return RTEOM_ERR_ARG; }
  rteom_status st = check_sizes(n_orb, n_occ_a, n_occ_b, n_chol, core_orb, core_spin, &m);
  if (st != RTEOM_OK) { g_last_error = m; return st; }
  rteom_options o;
  rteom_default_options(&o);
  if (opt) o = *opt;
  if (!valid_options(&o, &m)) { g_last_error = m; return RTEOM_ERR_ARG; }
  PlanResult r;
  st = choose_plan(n_orb, n_occ_a, n_occ_b, n_chol, core_orb, core_spin, o, &r);
  if (st == RTEOM_OK) *bytes = r.bytes;
  return st;
}

rteom_status rteom_init(rteom_ctx** out, int32_t n_orb, int32_t n_occ_a, int32_t n_occ_b,
                        const double* fock_diag, int32_t n_chol, const double* chol,
                        int32_t core_orb, int32_t core_spin, const rteom_options* opt) {
  std::string m;
  if (!out || !fock_diag || !chol) { g_last_error = "NULL argument"; return RTEOM_ERR_ARG; }
  *out = nullptr;
  rteom_status st = check_sizes(n_orb, n_occ_a, n_occ_b, n_chol, core_orb, core_spin, &m);
  if (st != RTEOM_OK) { g_last_error = m; return st; }
  rteom_options o;
  rteom_default_options(&o);
  if (opt) o = *opt;
  if (!valid_options(&o, &m)) { g_last_error = m; return RTEOM_ERR_ARG; }
  // inputs: finite, L symmetric
  for (int p = 0; p < n_orb; ++p)
    if (!std::isfinite(fock_diag[p])) { g_last_error = "non-finite orbital energy"; return RTEOM_ERR_NONFINITE; }
  const size_t nn = (size_t)n_orb * n_orb;
  double lmax = 0.0;
  for (size_t k = 0; k < (size_t)n_chol * nn; ++k) {
    if (!std::isfinite(chol[k])) { g_last_error = "non-finite Cholesky vector element"; return RTEOM_ERR_NONFINITE; }
    lmax = std::max(lmax, std::fabs(chol[k]));
  }
  for (int32_t q = 0; q < n_chol; ++q)
    for (int p = 0; p < n_orb; ++p)
      for (int r = 0; r < p; ++r) {
        double a = chol[q * nn + (size_t)p * n_orb + r], b = chol[q * nn + (size_t)r * n_orb + p];
        if (std::fabs(a - b) > 1e-12 * std::max(1.0, lmax)) {
          g_last_error = "Cholesky vectors are not symmetric in (p, q)";
          return RTEOM_ERR_ARG;
        }
      }
  PlanResult pr;
  st = choose_plan(n_orb, n_occ_a, n_occ_b, n_chol, core_orb, core_spin, o, &pr);
  if (st != RTEOM_OK) return st;
  const size_t need = pr.bytes;
  std::unique_ptr<rteom_ctx> ctx(new rteom_ctx());
  Context& c = ctx->c;
  c.opt = o;
  c.plan = pr.plan;
  c.res_flops = pr.flops;         // known from the plan before the first evaluation
  c.res_alg_flops = pr.alg_flops;
  for (int k = 0; k < rteom::kNumPhases; ++k) {
    c.res_phase_flops[k] = pr.phase_flops[k];
    c.res_alg_phase_flops[k] = pr.alg_phase_flops[k];
  }
  c.n = n_orb; c.nq = n_chol; c.na = n_occ_a; c.nb = n_occ_b; c.core_orb = core_orb; c.core_spin = core_spin;
  std::string berr;
#ifdef RTEOM_HOST_BACKEND
  c.be = rteom::make_host_backend();
#else
  c.be = rteom::make_hip_backend(o.stream, &berr);
#endif
  if (!c.be) { g_last_error = "backend: " + berr; return RTEOM_ERR_HIP; }
  if (o.workspace) {
    if (o.workspace_bytes < need) {
      g_last_error = "workspace too small: need " + std::to_string(need) + " bytes";
      delete c.be;
      c.be = nullptr;
      return RTEOM_ERR_OOM;
    }
    c.ws = o.workspace;
    c.arena.init(static_cast<char*>(c.ws), o.workspace_bytes);
  } else {
    c.ws = c.be->alloc(need);
    if (!c.ws) {
      g_last_error = "device allocation of " + std::to_string(need) + " bytes failed";
      delete c.be;
      c.be = nullptr;
      return RTEOM_ERR_OOM;
    }
    c.ws_owned = true;
    c.arena.init(static_cast<char*>(c.ws), need);
  }
  c.be->set_tuning(o.tune);
  st = guarded(ctx.get(), [&] {
    c.init(fock_diag, chol);
    // Graph-captured steps cannot time GEMM tile shapes: tune them now on one
    // residual evaluation (at T = 0; only shapes matter), outside any capture.
    // The same residual writes the resident converted integral blocks of the
    // reduced precisions, so that no captured graph holds their conversion.
    if ((o.tune || o.prec != RTEOM_FP64) && c.graph_mode()) {
      c.residual(c.X, c.R);
      c.be->sync();
    }
  });
  if (st != RTEOM_OK) {
    g_last_error = c.err;
    if (c.ws_owned) c.be->release(c.ws);
    delete c.be;
    c.be = nullptr;
    return st;
  }
  *out = ctx.release();
  return RTEOM_OK;
}

rteom_status rteom_step(rteom_ctx* ctx, double dt, int32_t n_steps, int32_t* iters) {
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  if (c.failed) { c.err = "context is in a failed state"; return RTEOM_ERR_STATE; }
  if (!(dt > 0.0) || !std::isfinite(dt) || n_steps < 0) { c.err = "dt must be positive and finite, n_steps >= 0"; return RTEOM_ERR_ARG; }
  rteom_status st = guarded(ctx, [&] {
    for (int32_t k = 0; k < n_steps; ++k) {
      int p = c.graph_mode() ? c.step_graphed(dt) : c.step(dt);
      if (iters) iters[k] = p;
    }
    c.be->sync();
    c.check_finite();
  });
  // a tolerance-driven step that failed left T and C(t) at the last committed step;
  // anything else that fails leaves the context unusable until it is reset
  if (st == RTEOM_ERR_HIP || ((st == RTEOM_ERR_NOCONV || st == RTEOM_ERR_NONFINITE) && !c.restored)) c.failed = true;
  return st;
}

rteom_status rteom_cumulant(const rteom_ctx* cctx, int64_t cap, double* t_out, double* c_out, int64_t* n_out) {
  rteom_ctx* ctx = const_cast<rteom_ctx*>(cctx);
  if (!ctx || !n_out || cap < 0) { g_last_error = "bad argument"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  return guarded(ctx, [&] {
    if (cap == 0) {  // length query
      *n_out = c.nsteps + 1;
      return;
    }
    int64_t n = std::min<int64_t>(cap, c.nsteps + 1);
    if (c_out && n > 0) c.be->d2h(c_out, c.c_hist, sizeof(double) * 2 * n);
    if (t_out)
      for (int64_t k = 0; k < n; ++k) t_out[k] = c.times[k];
    *n_out = n;
  });
}

namespace {
constexpr uint64_t kImageMagic = 0x4d4f4554522d5452ull;   // "RT-RTEOM" little-endian
constexpr uint32_t kImageVersion = 2;   // 2: same-spin doubles in pair storage
struct ImageHeader {
  uint64_t magic;
  uint32_t version, reserved;
  int32_t n_orb, n_occ_a, n_occ_b, n_chol, core_orb, core_spin;
  int64_t nsteps, amp_doubles;
};
size_t image_bytes(int64_t nsteps, int64_t amp_doubles) {
  // times, C history, E history, planar amplitudes
  return sizeof(ImageHeader) + sizeof(double) * (size_t)((nsteps + 1) * 5 + amp_doubles);
}
}  // namespace

rteom_status rteom_checkpoint(rteom_ctx* ctx, void* buf, size_t cap, size_t* bytes) {
  if (!ctx || !bytes) { g_last_error = "NULL argument"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  if (c.failed) { c.err = "context is in a failed state"; return RTEOM_ERR_STATE; }
  const int64_t amp = 2 * c.lay.size();
  *bytes = image_bytes(c.nsteps, amp);
  if (!buf) return RTEOM_OK;
  if (cap < *bytes) { c.err = "checkpoint buffer too small"; return RTEOM_ERR_ARG; }
  return guarded(ctx, [&] {
    ImageHeader h{};
    h.magic = kImageMagic;
    h.version = kImageVersion;
    h.n_orb = c.n; h.n_occ_a = c.na; h.n_occ_b = c.nb; h.n_chol = c.nq;
    h.core_orb = c.core_orb; h.core_spin = c.core_spin;
    h.nsteps = c.nsteps;
    h.amp_doubles = amp;
    char* p = static_cast<char*>(buf);
    std::memcpy(p, &h, sizeof(h));
    double* d = reinterpret_cast<double*>(p + sizeof(h));
    const int64_t n = c.nsteps + 1;
    for (int64_t k = 0; k < n; ++k) d[k] = c.times[k];
    c.be->d2h(d + n, c.c_hist, sizeof(double) * 2 * n);
    c.be->d2h(d + 3 * n, c.e_hist, sizeof(double) * 2 * n);
    c.be->d2h(d + 5 * n, c.X, sizeof(double) * amp);
  });
}

rteom_status rteom_restore(rteom_ctx* ctx, const void* buf, size_t len) {
  if (!ctx || !buf) { g_last_error = "NULL argument"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  ImageHeader h{};
  if (len < sizeof(h)) { c.err = "checkpoint image truncated"; return RTEOM_ERR_ARG; }
  std::memcpy(&h, buf, sizeof(h));
  const int64_t amp = 2 * c.lay.size();
  if (h.magic != kImageMagic || h.version != kImageVersion) { c.err = "not a checkpoint image"; return RTEOM_ERR_ARG; }
  if (h.n_orb != c.n || h.n_occ_a != c.na || h.n_occ_b != c.nb || h.n_chol != c.nq || h.core_orb != c.core_orb ||
      h.core_spin != c.core_spin || h.amp_doubles != amp) {
    c.err = "checkpoint image is for another system";
    return RTEOM_ERR_ARG;
  }
  if (h.nsteps < 0 || h.nsteps > c.opt.max_steps) { c.err = "checkpoint has more steps than max_steps"; return RTEOM_ERR_ARG; }
  if (len < image_bytes(h.nsteps, amp)) { c.err = "checkpoint image truncated"; return RTEOM_ERR_ARG; }
  const double* d = reinterpret_cast<const double*>(static_cast<const char*>(buf) + sizeof(h));
  const int64_t n = h.nsteps + 1;
  for (int64_t k = 0; k < 2 * n; ++k)
    if (!std::isfinite(d[n + k]) || !std::isfinite(d[3 * n + k])) { c.err = "non-finite history"; return RTEOM_ERR_NONFINITE; }
  for (int64_t k = 0; k < amp; ++k)
    if (!std::isfinite(d[5 * n + k])) { c.err = "non-finite amplitude"; return RTEOM_ERR_NONFINITE; }
  return guarded(ctx, [&] {
    c.be->h2d(c.c_hist, d + n, sizeof(double) * 2 * n);
    c.be->h2d(c.e_hist, d + 3 * n, sizeof(double) * 2 * n);
    c.be->h2d(c.X, d + 5 * n, sizeof(double) * amp);
    const int64_t step = h.nsteps;
    c.be->h2d(c.dstep, &step, sizeof(step));
    c.be->fill(c.dbad, 1, 0.0);
    c.nsteps = h.nsteps;
    c.times.assign(d, d + n);
    c.failed = false;
    c.be->sync();
  });
}

rteom_status rteom_ground_state(rteom_ctx* ctx, double tol, int32_t max_iter, double* e_corr, int32_t* iters) {
  if (!ctx || !e_corr) { g_last_error = "NULL argument"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  if (!(tol > 0.0) || !std::isfinite(tol) || max_iter < 1) { c.err = "tol must be positive, max_iter >= 1"; return RTEOM_ERR_ARG; }
  int passes = 0;
  rteom_status st = guarded(ctx, [&] { passes = c.ground_state(tol, max_iter, e_corr); });
  if (iters) *iters = passes;
  if (st == RTEOM_ERR_NOCONV || st == RTEOM_ERR_NONFINITE || st == RTEOM_ERR_HIP) c.failed = true;
  else if (st == RTEOM_OK) c.failed = false;
  return st;
}

// Arguments of rteom_spectral and its allocation-free variant.
static bool spectral_args(Context& c, double e_corr, double eta, int64_t n_w, const double* omega, const double* a_out) {
  if (c.core_orb < 0) { c.err = "the context has no core hole"; return false; }
  if (!omega || !a_out || n_w < 1) { c.err = "omega and a_out are required, n_w >= 1"; return false; }
  if (!std::isfinite(e_corr) || !std::isfinite(eta) || eta < 0.0) {
    c.err = "e_corr must be finite and eta finite and >= 0";
    return false;
  }
  for (int64_t j = 0; j < n_w; ++j)
    if (!std::isfinite(omega[j])) { c.err = "non-finite frequency"; return false; }
  return true;
}

// Doubles of device memory the spectrum needs: times, frequencies, weighted G, A, peak.
static int64_t spectral_doubles(const Context& c, int64_t n_w) { return 3 * (c.nsteps + 1) + 2 * n_w + 2; }

// The spectrum computed in the device buffer buf (spectral_doubles doubles).
static void spectral_into(Context& c, double* buf, double e_corr, double eta, int64_t n_w, const double* omega,
                          double* a_out, double* qp_out) {
  const int64_t n = c.nsteps + 1;
  double *t = buf, *w = t + n, *wg = w + n_w, *a = wg + 2 * n, *qp = a + n_w;
  c.be->h2d(t, c.times.data(), sizeof(double) * n);
  c.be->h2d(w, omega, sizeof(double) * n_w);
  c.be->spectral(c.c_hist, t, n, c.eps_core + e_corr, eta, w, n_w, wg, a, qp);
  c.be->d2h(a_out, a, sizeof(double) * n_w);
  if (qp_out) c.be->d2h(qp_out, qp, sizeof(double) * 2);
}

rteom_status rteom_spectral(rteom_ctx* ctx, double e_corr, double eta, int64_t n_w, const double* omega,
                            double* a_out, double* qp_out) {
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  if (!spectral_args(c, e_corr, eta, n_w, omega, a_out)) return RTEOM_ERR_ARG;
  return guarded(ctx, [&] {
    const size_t bytes = sizeof(double) * (size_t)spectral_doubles(c, n_w);
    std::unique_ptr<double, std::function<void(double*)>> buf(
        static_cast<double*>(c.be->alloc(bytes)), [&c](double* p) { if (p) c.be->release(p); });
    if (!buf) throw Error(RTEOM_ERR_OOM, "device allocation for the spectrum failed");
    spectral_into(c, buf.get(), e_corr, eta, n_w, omega, a_out, qp_out);
  });
}

rteom_status rteom_spectral_peaks(rteom_ctx* ctx, double e_corr, double eta, int64_t n_w, const double* omega,
                                  double* a_out, int32_t max_peaks, double* peaks_out, int32_t* n_peaks) {
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  std::vector<double> a_host;
  if (!a_out) {
    a_host.assign(n_w > 0 ? n_w : 1, 0.0);
    a_out = a_host.data();
  }
  if (!spectral_args(c, e_corr, eta, n_w, omega, a_out)) return RTEOM_ERR_ARG;
  if (max_peaks < 1 || max_peaks > 64 || !peaks_out || !n_peaks) {
    c.err = "max_peaks must be in 1..64, peaks_out and n_peaks are required";
    return RTEOM_ERR_ARG;
  }
  return guarded(ctx, [&] {
    const int64_t need = spectral_doubles(c, n_w) + 2 * max_peaks + 1;
    std::unique_ptr<double, std::function<void(double*)>> buf(
        static_cast<double*>(c.be->alloc(sizeof(double) * need)), [&c](double* p) { if (p) c.be->release(p); });
    if (!buf) throw Error(RTEOM_ERR_OOM, "device allocation for the spectrum failed");
    spectral_into(c, buf.get(), e_corr, eta, n_w, omega, a_out, nullptr);
    const int64_t n = c.nsteps + 1;
    double* a = buf.get() + n + n_w + 2 * n;        // A(omega) as spectral_into left it
    double* w = buf.get() + n;
    double* pk = buf.get() + spectral_doubles(c, n_w);
    c.be->spectral_peaks(a, w, n_w, max_peaks, pk);
    std::vector<double> host(2 * max_peaks + 1);
    c.be->d2h(host.data(), pk, sizeof(double) * host.size());
    *n_peaks = (int32_t)host[2 * max_peaks];
    for (int32_t q = 0; q < 2 * *n_peaks; ++q) peaks_out[q] = host[q];
  });
}

rteom_status rteom_spectral_noalloc(rteom_ctx* ctx, double e_corr, double eta, int64_t n_w, const double* omega,
                                    double* a_out, double* qp_out) {
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  if (!spectral_args(c, e_corr, eta, n_w, omega, a_out)) return RTEOM_ERR_ARG;
  int64_t cap = 0;
  double* buf = c.be->fixed_scratch(&cap);
  if (!buf) { c.err = "this backend has no fixed device scratch"; return RTEOM_ERR_STATE; }
  const int64_t need = spectral_doubles(c, n_w);
  if (need > cap) {
    c.err = "the spectrum needs " + std::to_string(need) + " doubles of fixed scratch (3 (steps + 1) + 2 n_w + 2), "
            "more than its " + std::to_string(cap);
    return RTEOM_ERR_ARG;
  }
  return guarded(ctx, [&] { spectral_into(c, buf, e_corr, eta, n_w, omega, a_out, qp_out); });
}

rteom_status rteom_dims(const rteom_ctx* cctx, int32_t* n_o, int32_t* n_v, int32_t* occ_list, int32_t* vir_list) {
  if (!cctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  const Context& c = cctx->c;
  if (n_o) *n_o = c.no;
  if (n_v) *n_v = c.nv;
  if (occ_list) for (int i = 0; i < c.no; ++i) occ_list[i] = c.O[i];
  if (vir_list) for (int a = 0; a < c.nv; ++a) vir_list[a] = c.V[a];
  return RTEOM_OK;
}

static void to_planar(const rteom::Context& c, const double* t1, const double* t2, std::vector<double>& buf) {
  const int64_t ns = c.lay.size(), n1 = 2 * c.lay.n1();
  buf.assign(2 * ns, 0.0);
  for (int64_t k = 0; k < n1; ++k) {
    buf[k] = t1 ? t1[2 * k] : 0.0;
    buf[ns + k] = t1 ? t1[2 * k + 1] : 0.0;
  }
  for (int64_t k = 0; k < ns - n1; ++k) {
    buf[n1 + k] = t2 ? t2[2 * k] : 0.0;
    buf[ns + n1 + k] = t2 ? t2[2 * k + 1] : 0.0;
  }
}

static void from_planar(const rteom::Context& c, const std::vector<double>& buf, double* t1, double* t2) {
  const int64_t ns = c.lay.size(), n1 = 2 * c.lay.n1();
  if (t1)
    for (int64_t k = 0; k < n1; ++k) {
      t1[2 * k] = buf[k];
      t1[2 * k + 1] = buf[ns + k];
    }
  if (t2)
    for (int64_t k = 0; k < ns - n1; ++k) {
      t2[2 * k] = buf[n1 + k];
      t2[2 * k + 1] = buf[ns + n1 + k];
    }
}

rteom_status rteom_set_amplitudes(rteom_ctx* ctx, const double* t1, const double* t2) {
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  return guarded(ctx, [&] {
    if (t1 || t2) {
      std::vector<double> buf;
      to_planar(c, t1, t2, buf);
      for (double v : buf)
        if (!std::isfinite(v)) throw Error(RTEOM_ERR_NONFINITE, "non-finite amplitude");
      c.be->h2d(c.X, buf.data(), buf.size() * sizeof(double));
    }
    c.mask_set(c.X);
    c.energy(c.X, c.e_hist + 2 * c.nsteps);   // E(T_n) for the next trapezoid
    c.be->fill(c.dbad, 1, 0.0);
    c.failed = false;
  });
}

rteom_status rteom_device_sets(const rteom_ctx* cctx, void** x, void** r, int64_t* doubles) {
  if (!cctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  const Context& c = cctx->c;
  if (x) *x = c.X;
  if (r) *r = c.R;
  if (doubles) *doubles = 2 * c.lay.size();
  return RTEOM_OK;
}

rteom_status rteom_get_amplitudes(const rteom_ctx* cctx, double* t1, double* t2) {
  rteom_ctx* ctx = const_cast<rteom_ctx*>(cctx);
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  return guarded(ctx, [&] {
    std::vector<double> buf(2 * c.lay.size());
    c.be->d2h(buf.data(), c.X, buf.size() * sizeof(double));
    from_planar(c, buf, t1, t2);
  });
}

rteom_status rteom_residual(rteom_ctx* ctx, double* r1, double* r2) {
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  return guarded(ctx, [&] {
    c.residual(c.X, c.R);
    if (r1 || r2) {
      std::vector<double> buf(2 * c.lay.size());
      c.be->d2h(buf.data(), c.R, buf.size() * sizeof(double));
      from_planar(c, buf, r1, r2);
    } else {
      c.be->sync();
    }
  });
}

rteom_status rteom_energy(rteom_ctx* ctx, double* e_out) {
  if (!ctx || !e_out) { g_last_error = "bad argument"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  return guarded(ctx, [&] {
    double* tmp = c.delta;  // reuse: energy is written to the e_hist slot of the current step
    (void)tmp;
    const size_t mk = c.arena.mark();
    double* e = c.arena.take(2);
    c.energy(c.X, e);
    c.be->d2h(e_out, e, 2 * sizeof(double));
    c.arena.release(mk);
  });
}

rteom_status rteom_residual_flops(const rteom_ctx* cctx, double* flops) {
  if (!cctx || !flops) { g_last_error = "bad argument"; return RTEOM_ERR_ARG; }
  *flops = cctx->c.res_alg_flops;
  return RTEOM_OK;
}

rteom_status rteom_plan_info(const rteom_ctx* cctx, int32_t* resident, int64_t* e_slab, int64_t* ring_cols,
                             int64_t* rows, double* exec_flops, size_t* workspace_bytes) {
  if (!cctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  const Context& c = cctx->c;
  if (resident) *resident = c.plan.resident ? 1 : 0;
  if (e_slab) *e_slab = c.plan.resident ? c.nv : std::min<int64_t>(c.plan.es, c.nv);
  if (ring_cols) *ring_cols = std::min<int64_t>(c.plan.cj, c.no);
  if (rows) *rows = std::min<int64_t>(c.plan.ci, c.no);
  if (exec_flops) *exec_flops = c.res_flops;
  if (workspace_bytes) *workspace_bytes = c.arena.capacity();
  return RTEOM_OK;
}

rteom_status rteom_profile(rteom_ctx* ctx, uint32_t phase_mask) {
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  ctx->c.be->set_profile(phase_mask);
  return RTEOM_OK;
}

// Tile-choice cache file: a header line "rteom-tiles 1 <arch>", then one line per timed
// GEMM signature: the ten key values and the tile shape, as decimal integers.
static const char kTileMagic[] = "rteom-tiles";

rteom_status rteom_tile_cache_save(rteom_ctx* ctx, const char* path) {
  if (!ctx || !path) { g_last_error = "NULL argument"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  return guarded(ctx, [&] {
    constexpr int w = rteom::Backend::kTileKey + 1;
    const int64_t n = c.be->tile_table(nullptr, 0);
    std::vector<int64_t> rows((size_t)std::max<int64_t>(1, n) * w);
    c.be->tile_table(rows.data(), n);
    std::FILE* f = std::fopen(path, "w");
    if (!f) throw Error(RTEOM_ERR_ARG, std::string("cannot write ") + path);
    bool ok = std::fprintf(f, "%s 1 %s\n", kTileMagic, c.be->device_arch().c_str()) > 0;
    for (int64_t i = 0; i < n && ok; ++i) {
      for (int k = 0; k < w && ok; ++k)
        ok = std::fprintf(f, k + 1 < w ? "%lld " : "%lld\n", (long long)rows[(size_t)(i * w + k)]) > 0;
    }
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) throw Error(RTEOM_ERR_ARG, std::string("write error on ") + path);
  });
}

rteom_status rteom_tile_cache_load(rteom_ctx* ctx, const char* path) {
  if (!ctx || !path) { g_last_error = "NULL argument"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  return guarded(ctx, [&] {
    constexpr int w = rteom::Backend::kTileKey + 1;
    std::FILE* f = std::fopen(path, "r");
    if (!f) throw Error(RTEOM_ERR_ARG, std::string("cannot read ") + path);
    char magic[32] = {0}, arch[128] = {0};
    int version = 0;
    const int got = std::fscanf(f, "%31s %d %127s", magic, &version, arch);
    if (got != 3 || std::strcmp(magic, kTileMagic) != 0 || version != 1) {
      std::fclose(f);
      throw Error(RTEOM_ERR_ARG, std::string(path) + " is not a tile cache file");
    }
    if (c.be->device_arch() != arch) {
      std::fclose(f);
      throw Error(RTEOM_ERR_ARG, std::string(path) + " holds tile choices for " + arch + ", not for " +
                                     c.be->device_arch());
    }
    std::vector<int64_t> rows;
    long long v = 0;
    int r;
    while ((r = std::fscanf(f, "%lld", &v)) == 1) rows.push_back(v);
    const bool eof = std::feof(f) != 0;
    std::fclose(f);
    if (r != EOF || !eof || rows.size() % w != 0)
      throw Error(RTEOM_ERR_ARG, std::string(path) + ": malformed tile cache entries");
    std::string m;
    if (!c.be->load_tile_table(rows.data(), (int64_t)(rows.size() / w), &m)) throw Error(RTEOM_ERR_ARG, path + (": " + m));
  });
}

rteom_status rteom_phase_stats(rteom_ctx* ctx, int32_t phase, double* ms, double* flops, int64_t* ops) {
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  if (phase < 0 || phase >= rteom::kNumPhases) { ctx->c.err = "bad phase"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  return guarded(ctx, [&] {
    int64_t n = 0;
    const double t = c.be->phase_ms(phase, &n);
    if (ms) *ms = t;
    if (ops) *ops = n;
    if (flops) *flops = c.res_alg_phase_flops[phase];
  });
}

struct rteom_batch {
  std::vector<rteom_ctx*> ctxs;
  std::string err;
};

rteom_status rteom_batch_create(rteom_batch** out, int32_t n, rteom_ctx* const* ctxs) {
  if (!out || n < 1 || !ctxs) { g_last_error = "bad argument"; return RTEOM_ERR_ARG; }
  *out = nullptr;
  for (int32_t k = 0; k < n; ++k) {
    if (!ctxs[k]) { g_last_error = "NULL context in batch"; return RTEOM_ERR_ARG; }
    const Context& c = ctxs[k]->c;
    if (!c.graph_mode()) { g_last_error = "batched contexts need graph mode and fixed passes"; return RTEOM_ERR_STATE; }
    if (c.failed) { g_last_error = "context in a failed state"; return RTEOM_ERR_STATE; }
    for (int32_t j = 0; j < k; ++j)
      if (ctxs[j] == ctxs[k]) { g_last_error = "context listed twice"; return RTEOM_ERR_ARG; }
  }
  rteom_batch* b = new rteom_batch();
  b->ctxs.assign(ctxs, ctxs + n);
  *out = b;
  return RTEOM_OK;
}

rteom_status rteom_batch_step(rteom_batch* b, double dt, int32_t n_steps) {
  if (!b) { g_last_error = "NULL batch"; return RTEOM_ERR_ARG; }
  if (!(dt > 0.0) || !std::isfinite(dt) || n_steps < 0) { b->err = "bad dt or n_steps"; g_last_error = b->err; return RTEOM_ERR_ARG; }
  rteom_ctx* lead = b->ctxs[0];
  rteom_status st = guarded(lead, [&] {
    for (rteom_ctx* x : b->ctxs)
      if (x->c.nsteps + n_steps > x->c.opt.max_steps) throw Error(RTEOM_ERR_STATE, "C(t) history would overflow");
    // Every member's captured step is replayed on the member's own stream, all members
    // before any wait: the streams map onto the device's hardware queues, so the small
    // products of different members run side by side.  (One parent graph holding every
    // member's step as a child node ran them one after another on this runtime.)
    for (rteom_ctx* x : b->ctxs)
      if (!x->c.graph_for(dt)) throw Error(RTEOM_ERR_STATE, "graph capture unavailable (null stream?)");
    for (rteom_ctx* x : b->ctxs) x->c.be->sync();
    for (int32_t k = 0; k < n_steps; ++k) {
      for (rteom_ctx* x : b->ctxs) {
        x->c.be->launch_graph(x->c.graph_for(dt));
        ++x->c.nsteps;
        x->c.times.push_back(x->c.times.back() + dt);
      }
    }
    for (rteom_ctx* x : b->ctxs) x->c.be->sync();
    for (size_t k = 0; k < b->ctxs.size(); ++k) {
      Context& x = b->ctxs[k]->c;
      try {
        x.check_finite();
      } catch (const Error& e) {
        x.failed = true;
        x.err = e.what();
        throw Error(e.code, "batch member " + std::to_string(k) + ": " + e.what());
      }
    }
  });
  if (st != RTEOM_OK) g_last_error = lead->c.err;
  return st;
}

rteom_status rteom_batch_free(rteom_batch* b) {
  if (!b) return RTEOM_OK;
  delete b;
  return RTEOM_OK;
}

rteom_status rteom_free(rteom_ctx* ctx) {
  if (!ctx) return RTEOM_OK;
  Context& c = ctx->c;
  if (c.be) {
    c.be->sync();
    if (c.step_graph) c.be->destroy_graph(c.step_graph);
    if (c.ws_owned && c.ws) c.be->release(c.ws);
    delete c.be;
  }
  delete ctx;
  return RTEOM_OK;
}

const char* rteom_last_error(const rteom_ctx* ctx) {
  return ctx ? ctx->c.err.c_str() : g_last_error.c_str();
}

}  // extern "C"
