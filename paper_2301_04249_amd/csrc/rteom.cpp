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
//   (aa, ab, bb) share one shape and one set of integral blocks.
// * Residual.  R_x = <Phi_x| e^{-T} H_N e^{T} |Phi> is evaluated in the
//   T1-similarity-transformed ("dressed") form: e^{-T1} H e^{T1} has the
//   Cholesky vectors L~ = (1 - t) L (1 + t) (t: the virtual-by-occupied T1
//   matrix) and the dressed Fock matrix f~ = (1 - t) h (1 + t) + J~ - K~ of Phi,
//   and R is the CCD-like projection of that Hamiltonian with T2 (Eqs. dt1eom,
//   dt2eom).  The pp-ladder keeps the real (ae|bf) integrals; the T1 part of the
//   dressed virtual vectors becomes the o^3 v^3 "Z" terms and an o^4 v^2 term.
//   Coulomb-type ring terms are factorised through D^Q_ia = sum_me T_imae L^Q_me.
// * Step.  Implicit trapezoid (Eq. trapzrule) with fixed-point passes; three
//   amplitude-sized buffers (iterate X, rhs, residual R) as in Table 2's three
//   timeline tensors.  C(t) accumulates i E(T) with the same trapezoid weights.
#include <algorithm>
#include <cmath>
#include <complex>
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

  int n = 0, nq = 0, na = 0, nb = 0, core_orb = 0, core_spin = 0;
  int no = 0, nv = 0, nx = 0;
  std::vector<int> O, V;
  std::vector<double> mo_h[2], mv_h[2];
  AmpLayout lay;

  double* mo[2] = {nullptr, nullptr};
  double* mv[2] = {nullptr, nullptr};
  double* fo[2] = {nullptr, nullptr};
  double* fv[2] = {nullptr, nullptr};
  double *Loo = nullptr, *Lov = nullptr, *Lvv = nullptr, *Lvo = nullptr;
  double* f[2] = {nullptr, nullptr};   // undressed Fock of Phi, [nx][nx]
  double* h[2] = {nullptr, nullptr};   // one-body part h = f - G, [nx][nx]
  double* Jov = nullptr;               // (me|nf) as [m][e][n][f]
  double* Vlad = nullptr;              // (ae|bf) as [e][f][a][b]
  double* B1 = nullptr;                // (me|bf) as [e][f][m][b]
  // Same-spin blocks in antisymmetric pair storage (pairs e < f, a < b in
  // lexicographic order): <ab||ef> = (ae|bf) - (af|be) as [ef][ab], and
  // (me|bf) - (mf|be) as [ef][m][b]
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
  double res_flops = 0.0;
  double res_phase_flops[kNumPhases] = {0};

  // ---------------------------------------------------------------- views
  View Lv(double* p, int64_t a, int64_t b) const { return make_view(p, nullptr, {nq, a, b}); }
  View t1(double* set, int s) const {
    return make_view(set + s * lay.n1(), set + lay.size() + s * lay.n1(), {no, nv});
  }
  View t2(double* set, int b) const {
    double* p = set + 2 * lay.n1() + b * lay.n2();
    return make_view(p, p + lay.size(), {no, no, nv, nv});
  }
  // spin-aligned doubles block t_{i s, m u}^{a s, e u} as a [i][m][a][e] view
  View TT(double* set, int s, int u) const {
    if (s == u) return t2(set, s == 0 ? 0 : 2);
    View ab = t2(set, 1);
    return s == 0 ? ab : reorder(ab, {1, 0, 3, 2});
  }
  View fview(double* p, int64_t r0, int64_t c0, int64_t nr, int64_t nc, bool cplx) const {
    View v = make_view(p, cplx ? p + (int64_t)nx * nx : nullptr, {nx, nx});
    return block(v, {r0, c0}, {nr, nc});
  }
  View vec(double* p, int64_t n) const { return make_view(p, nullptr, {n}); }
  static int64_t npairs(int64_t n) { return n * (n - 1) / 2; }
  // the two same-spin doubles blocks (0: alpha alpha, 2: beta beta) of a set and
  // a packed [2][pairs (i<j)][...] array
  PairOp same_spin_pairs(double* set_blocks, const View& packed, int64_t n2, int pair2) const {
    PairOp op;
    op.n1 = no; op.n2 = n2; op.nblk = 2; op.pair2 = pair2;
    op.x_re = set_blocks; op.x_im = set_blocks + lay.size(); op.x_bs = 2 * lay.n2();
    op.y_re = packed.re; op.y_im = packed.im; op.y_bs = packed.numel() / 2;
    return op;
  }

  double* take(int64_t n) { return arena.take(n); }
  void h2d(double* dst, const double* src, int64_t n) {
    if (!dry) be->h2d(dst, src, n * sizeof(double));
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
      for (int i = 0; i < no; ++i) mo_h[s][i] = occ[s][O[i]];
      for (int a = 0; a < nv; ++a) mv_h[s][a] = vir[s][V[a]];
    }
    lay.no = no;
    lay.nv = nv;
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
    Loo = take(Q * no * no);
    Lov = take(Q * no * nv);
    Lvv = take(Q * nv * nv);
    Lvo = take(Q * nv * no);
    Jov = take((int64_t)no * nv * no * nv);
    Vlad = take((int64_t)nv * nv * nv * nv);
    B1 = take((int64_t)nv * nv * no * nv);
    Wpp = take(npairs(nv) * npairs(nv));
    B1p = take(npairs(nv) * no * nv);
    if (opt.prec != RTEOM_FP64) {
      const int64_t v2 = (int64_t)nv * nv, pv = npairs(nv), ov = (int64_t)no * nv;
      const std::pair<ConvSlot*, int64_t> slots[4] = {
          {&conv_v, conv_doubles(v2, v2)}, {&conv_w, conv_doubles(pv, pv)},
          {&conv_b1, conv_doubles(ov, v2)}, {&conv_b1p, conv_doubles(ov, pv)}};
      for (const auto& sl : slots) {
        *sl.first = ConvSlot();
        sl.first->doubles = sl.second;
        sl.first->p = take(sl.second);
      }
    }
    const int64_t ns = lay.size();
    X = take(2 * ns);
    RHS = take(2 * ns);
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
    // Resident integral blocks (spin free)
    eng.contract("Qme,Qnf->menf", Lv(Lov, no, nv), Lv(Lov, no, nv),
                 make_view(Jov, nullptr, {no, nv, no, nv}), 1.0, 0);
    // (ae|bf) and (me|bf) are built in slabs of e: the product lands in a temporary
    // in GEMM order before it is permuted into place, and a slab bounds that
    // temporary to kSlabDoubles instead of a second copy of the whole block.
    {
      const int64_t per_e = std::max<int64_t>(1, (int64_t)nv * nv * nv);
      const int64_t ce = std::max<int64_t>(1, std::min<int64_t>(nv, kSlabDoubles / per_e));
      View Vv = make_view(Vlad, nullptr, {nv, nv, nv, nv});
      View Bv = make_view(B1, nullptr, {nv, nv, no, nv});
      for (int64_t e0 = 0; e0 < nv; e0 += ce) {
        const int64_t n = std::min<int64_t>(ce, nv - e0);
        View Le = block(Lv(Lvv, nv, nv), {0, 0, e0}, {Q, nv, n});
        View Lm = block(Lv(Lov, no, nv), {0, 0, e0}, {Q, no, n});
        eng.contract("Qae,Qbf->efab", Le, Lv(Lvv, nv, nv), block(Vv, {e0, 0, 0, 0}, {n, nv, nv, nv}), 1.0, 0);
        eng.contract("Qme,Qbf->efmb", Lm, Lv(Lvv, nv, nv), block(Bv, {e0, 0, 0, 0}, {n, nv, no, nv}), 1.0, 0);
      }
    }
    {
      PairOp w;
      w.n1 = nv; w.n2 = nv; w.pair2 = 1; w.anti = 1;
      w.x_re = Vlad; w.y_re = Wpp;
      eng.pairs(w);
      PairOp z;
      z.n1 = nv; z.n2 = (int64_t)no * nv; z.pair2 = 0; z.anti = 1;
      z.x_re = B1; z.y_re = B1p;
      eng.pairs(z);
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
  // R <- <Phi_x| e^{-T} H_N e^{T} |Phi> for T = Xs (all five blocks, masked).
  void residual(double* Xs, double* Rs) {
    const int64_t Q = nq;
    const size_t mk = arena.mark();
    eng.prec = opt.prec;     // the residual's contractions in the requested precision
    eng.flops = 0.0;
    for (double& f : eng.phase_flops) f = 0.0;
    eng.set_phase(kPhaseGemm);
    View Lov_v = Lv(Lov, no, nv);
    View Ldoo[2], Ldvv[2], Ldvo[2], fd[2], D[2], Lbar[2], Fvv[2], Foo[2];
    // dressed Cholesky vectors L~ = (1 - t) L (1 + t)
    for (int s = 0; s < 2; ++s) {
      View t = t1(Xs, s);
      Ldoo[s] = eng.temp({Q, no, no}, true);
      eng.add(Ldoo[s], Lv(Loo, no, no), 1, 0, 0);
      eng.contract("Qmf,if->Qmi", Lov_v, t, Ldoo[s], 1.0, 1);
      Ldvv[s] = eng.temp({Q, nv, nv}, true);
      eng.add(Ldvv[s], Lv(Lvv, nv, nv), 1, 0, 0);
      eng.contract("ma,Qme->Qae", t, Lov_v, Ldvv[s], -1.0, 1);
      Ldvo[s] = eng.temp({Q, nv, no}, true);
      eng.add(Ldvo[s], Lv(Lvo, nv, no), 1, 0, 0);
      eng.contract("Qaf,if->Qai", Lv(Lvv, nv, nv), t, Ldvo[s], 1.0, 1);
      eng.contract("ma,Qmi->Qai", t, Ldoo[s], Ldvo[s], -1.0, 1);
    }
    // dressed Fock of Phi: f~ = (1 - t) h (1 + t) + J~ - K~
    View jq = eng.temp({Q}, true);
    for (int t = 0; t < 2; ++t)
      eng.contract("Qk,k->Q", diagonal(Ldoo[t], 1, 2), vec(mo[t], no), jq, 1.0, t);
    for (int s = 0; s < 2; ++s) {
      View t = t1(Xs, s);
      fd[s] = eng.temp({nx, nx}, true);
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
    }
    // D^Q_ia = sum_{me} T_imae L^Q_me summed over the spin of (m, e)
    for (int s = 0; s < 2; ++s) {
      D[s] = eng.temp({Q, no, nv}, true);
      eng.contract("imae,Qme->Qia", TT(Xs, s, s), Lov_v, D[s], 1.0, 0);
      eng.contract("imae,Qme->Qia", TT(Xs, s, 1 - s), Lov_v, D[s], 1.0, 1);
      Lbar[s] = eng.temp({Q, nv, no}, true);
      eng.add(Lbar[s], Ldvo[s], 1, 0, 0);
      eng.add(Lbar[s], reorder(D[s], {0, 2, 1}), 1, 0, 1);
      Fvv[s] = eng.temp({nv, nv}, true);
      eng.add(Fvv[s], fview(fd[s].re, no, no, nv, nv, true), 1, 0, 0);
      eng.contract("Qmb,Qme->be", D[s], Lov_v, Fvv[s], -1.0, 1);
      Foo[s] = eng.temp({no, no}, true);
      eng.add(Foo[s], fview(fd[s].re, 0, 0, no, no, true), 1, 0, 0);
      eng.contract("Qme,Qje->mj", Lov_v, D[s], Foo[s], 1.0, 1);
    }
    // singles
    for (int s = 0; s < 2; ++s) {
      const int u = 1 - s;
      View r1 = t1(Rs, s);
      eng.add(r1, reorder(fview(fd[s].re, no, 0, nv, no, true), {1, 0}), 1, 0, 0);
      eng.contract("me,imae->ia", fview(fd[s].re, 0, no, no, nv, true), TT(Xs, s, s), r1, 1.0, 1);
      eng.contract("me,imae->ia", fview(fd[u].re, 0, no, no, nv, true), TT(Xs, s, u), r1, 1.0, 1);
      eng.contract("Qae,Qie->ia", Ldvv[s], D[s], r1, 1.0, 1);
      eng.contract("Qmi,Qma->ia", Ldoo[s], D[s], r1, -1.0, 1);
      const double* sc[2] = {mo[s], mv[s]};
      eng.scale(r1, sc);
    }
    // ring intermediates W[(m,e),(b,j)]: exchange blocks WX(s,u) (m,j in s; b,e in u)
    // and the opposite-spin exchange blocks V(s->u) (m,e in s; j,b in u)
    View Jv = make_view(Jov, nullptr, {no, nv, no, nv});
    View WX[2][2], Vx[2];
    eng.set_phase(kPhaseRing);
    for (int s = 0; s < 2; ++s)
      for (int u = 0; u < 2; ++u) {
        WX[s][u] = eng.temp({no, nv, nv, no}, true);
        eng.contract("Qmj,Qbe->mbej", Ldoo[s], Ldvv[u], WX[s][u], -1.0, 0);
        eng.contract("jnfb,mfne->mbej", TT(Xs, s, u), Jv, WX[s][u], 0.5, 1);
      }
    for (int s = 0; s < 2; ++s) {
      const int u = 1 - s;
      Vx[s] = eng.temp({no, nv, nv, no}, true);
      eng.contract("jnbf,mfne->mbej", TT(Xs, u, s), Jv, Vx[s], -0.5, 0);
    }
    eng.set_phase(kPhaseGemm);
    View x = eng.temp({no, no, nv, nv}, true);
    View tau = eng.temp({no, no, nv, nv}, true);
    View g = eng.temp({no, no, no, no}, true);
    View gA = eng.temp({no, no, no, no}, true);
    View Xo = eng.temp({no, no, no, no}, true);
    View Vl = make_view(Vlad, nullptr, {nv, nv, nv, nv});
    View Bv = make_view(B1, nullptr, {nv, nv, no, nv});
    // all three doubles blocks are contiguous: [3 * no * no][nv][nv]
    const int64_t P3 = 3 * (int64_t)no * no;
    double* x2 = Xs + 2 * lay.n1();
    double* r2 = Rs + 2 * lay.n1();
    // same-spin doubles in pair storage [2][i<j][e<f] (T is antisymmetric in both pairs)
    const int64_t npo = npairs(no), npv = npairs(nv), nov = (int64_t)no * nv;
    View Tp = eng.temp({2 * npo, npv}, true);
    eng.pairs(same_spin_pairs(x2, Tp, nv, 1));
    View Tab = make_view(x2 + lay.n2(), x2 + lay.size() + lay.n2(), {(int64_t)no * no, nv, nv});
    View Rab = make_view(r2 + lay.n2(), r2 + lay.size() + lay.n2(), {(int64_t)no * no, nv, nv});
    // T1 part of the dressed virtual vectors ("Z" terms): Z_ij,mb = sum_ef T_ijef (me|bf),
    // for the same-spin blocks sum_{e<f} T_ijef [(me|bf) - (mf|be)] over pairs i < j
    View Z3 = eng.temp({P3, no, nv}, true);
    eng.set_phase(kPhaseRing);
    {
      const int64_t zb = (int64_t)no * no * nov;
      eng.contract("Pef,efmb->Pmb", Tab, Bv, make_view(Z3.re + zb, Z3.im + zb, {(int64_t)no * no, no, nv}), 1.0, 0,
                   &conv_b1);
      const size_t mz = arena.mark();
      View Zp = eng.temp({2 * npo, nov}, true);
      eng.contract("Pq,qc->Pc", Tp, make_view(B1p, nullptr, {npv, nov}), Zp, 1.0, 0, &conv_b1p);
      PairOp u;
      u.n1 = no; u.n2 = nov; u.nblk = 2; u.pair2 = 0; u.mode = 1; u.beta = 0;
      u.x_re = Z3.re; u.x_im = Z3.im; u.x_bs = 2 * zb;
      u.y_re = Zp.re; u.y_im = Zp.im; u.y_bs = npo * nov;
      eng.pairs(u);
      arena.release(mz);
    }
    eng.set_phase(kPhaseGemm);
    // same-spin doubles
    for (int s = 0; s < 2; ++s) {
      const int u = 1 - s;
      const int blk = s == 0 ? 0 : 2;
      View Rv = t2(Rs, blk), T = t2(Xs, blk), t = t1(Xs, s);
      // dressed <ab||ij> plus Coulomb ring: Lbar_ai Lbar_bj - Lbar_aj Lbar_bi
      eng.contract("Qai,Qbj->ijab", Lbar[s], Lbar[s], x, 1.0, 0);
      eng.add(Rv, x, 1, 0, 0);
      eng.add(Rv, reorder(x, {1, 0, 2, 3}), -1, 0, 1);
      eng.contract("ijae,be->ijab", T, Fvv[s], x, 1.0, 0);
      eng.add(Rv, x, 1, 0, 1);
      eng.add(Rv, reorder(x, {0, 1, 3, 2}), -1, 0, 1);
      eng.contract("imab,mj->ijab", T, Foo[s], x, 1.0, 0);
      eng.add(Rv, x, -1, 0, 1);
      eng.add(Rv, reorder(x, {1, 0, 2, 3}), 1, 0, 1);
      // hole ladder with the T1-T1 piece of the dressed particle ladder
      eng.contract("Qmi,Qnj->mnij", Ldoo[s], Ldoo[s], g, 1.0, 0);
      eng.add(gA, g, 1, 0, 0);
      eng.add(gA, reorder(g, {0, 1, 3, 2}), -1, 0, 1);
      eng.contract("ijef,menf->ijmn", T, Jv, Xo, 1.0, 0);
      eng.add(tau, T, 1, 0, 0);
      eng.contract("ia,jb->ijab", t, t, tau, 1.0, 1);
      eng.contract("ib,ja->ijab", t, t, tau, -1.0, 1);
      eng.contract("mnab,mnij->ijab", T, gA, Rv, 0.5, 1);
      eng.contract("mnab,ijmn->ijab", tau, Xo, Rv, 0.5, 1);
      // Z: -P(ab) sum_m t_ma Z_ij,mb
      View Zs = make_view(Z3.re + blk * (int64_t)no * no * no * nv, Z3.im + blk * (int64_t)no * no * no * nv,
                          {no, no, no, nv});
      eng.contract("ma,ijmb->ijab", t, Zs, x, -1.0, 0);
      eng.add(Rv, x, 1, 0, 1);
      eng.add(Rv, reorder(x, {0, 1, 3, 2}), -1, 0, 1);
      // exchange ring, P(ij) P(ab)
      eng.set_phase(kPhaseRing);
      eng.contract("imae,mbej->ijab", T, WX[s][s], x, 1.0, 0);
      eng.contract("imae,mbej->ijab", TT(Xs, s, u), Vx[u], x, 1.0, 1);
      eng.set_phase(kPhaseGemm);
      eng.add(Rv, x, 1, 0, 1);
      eng.add(Rv, reorder(x, {1, 0, 2, 3}), -1, 0, 1);
      eng.add(Rv, reorder(x, {0, 1, 3, 2}), -1, 0, 1);
      eng.add(Rv, reorder(x, {1, 0, 3, 2}), 1, 0, 1);
    }
    // alpha-beta doubles
    {
      View Rv = t2(Rs, 1), T = t2(Xs, 1);
      View ta = t1(Xs, 0), tb = t1(Xs, 1);
      eng.contract("Qai,Qbj->ijab", Lbar[0], Lbar[1], Rv, 1.0, 0);
      eng.contract("ijae,be->ijab", T, Fvv[1], Rv, 1.0, 1);
      eng.contract("ae,ijeb->ijab", Fvv[0], T, Rv, 1.0, 1);
      eng.contract("imab,mj->ijab", T, Foo[1], Rv, -1.0, 1);
      eng.contract("mi,mjab->ijab", Foo[0], T, Rv, -1.0, 1);
      eng.contract("Qmi,Qnj->mnij", Ldoo[0], Ldoo[1], g, 1.0, 0);
      eng.contract("ijef,menf->ijmn", T, Jv, Xo, 1.0, 0);
      eng.add(tau, T, 1, 0, 0);
      eng.contract("ia,jb->ijab", ta, tb, tau, 1.0, 1);
      eng.contract("mnab,mnij->ijab", T, g, Rv, 1.0, 1);
      eng.contract("mnab,ijmn->ijab", tau, Xo, Rv, 1.0, 1);
      View Zs = make_view(Z3.re + (int64_t)no * no * no * nv, Z3.im + (int64_t)no * no * no * nv, {no, no, no, nv});
      eng.contract("ma,ijmb->ijab", ta, Zs, Rv, -1.0, 1);
      View Z2 = eng.temp({no, no, nv, no}, true);
      eng.set_phase(kPhaseRing);
      eng.contract("ijef,fena->ijan", T, Bv, Z2, 1.0, 0);   // sum_ef T_ijef (ae|nf)
      eng.set_phase(kPhaseGemm);
      eng.contract("nb,ijan->ijab", tb, Z2, Rv, -1.0, 1);
      eng.set_phase(kPhaseRing);
      eng.contract("imae,mbej->ijab", T, WX[1][1], Rv, 1.0, 1);
      eng.contract("mjae,mbei->ijab", T, WX[0][1], Rv, 1.0, 1);
      eng.contract("imeb,maej->ijab", T, WX[1][0], Rv, 1.0, 1);
      eng.contract("mjeb,maei->ijab", T, WX[0][0], Rv, 1.0, 1);
      eng.contract("imae,mbej->ijab", t2(Xs, 0), Vx[0], Rv, 1.0, 1);
      eng.contract("jmbe,maei->ijab", t2(Xs, 2), Vx[1], Rv, 1.0, 1);
      eng.set_phase(kPhaseGemm);
    }
    // particle-particle ladder with the real (ae|bf): the alpha-beta block in full
    // storage, the same-spin blocks as sum_{e<f} T_ijef <ab||ef> over pairs i < j, a < b
    eng.set_phase(kPhaseLadder);
    eng.contract("Pef,efab->Pab", Tab, Vl, Rab, 1.0, 1, &conv_v);
    {
      const size_t mz = arena.mark();
      View Zp = eng.temp({2 * npo, npv}, true);
      eng.contract("Pq,qr->Pr", Tp, make_view(Wpp, nullptr, {npv, npv}), Zp, 1.0, 0, &conv_w);
      PairOp u = same_spin_pairs(r2, Zp, nv, 1);
      u.mode = 1;
      u.beta = 1;
      eng.pairs(u);
      arena.release(mz);
    }
    eng.set_phase(kPhaseGemm);
    // zero the amplitudes of spin-orbitals that do not exist
    {
      const int sp[3][2] = {{0, 0}, {0, 1}, {1, 1}};
      for (int b = 0; b < 3; ++b) {
        const double* sc[4] = {mo[sp[b][0]], mo[sp[b][1]], mv[sp[b][0]], mv[sp[b][1]]};
        eng.scale(t2(Rs, b), sc);
      }
    }
    res_flops = eng.flops;
    for (int k = 0; k < kNumPhases; ++k) res_phase_flops[k] = eng.phase_flops[k];
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
    u.x_re = X;
    u.x_im = X + lay.size();
    u.r_re = R;
    u.r_im = R + lay.size();
    u.rhs_re = RHS;
    u.rhs_im = RHS + lay.size();
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

  // Same-spin doubles are stored in full; keep them antisymmetric in a Jacobi
  // iteration, whose map amplifies their symmetric part (which the equations never
  // constrain) from rounding level by ~0.17 e-folds per iteration otherwise.
  void antisymmetrize_same_spin(double* set) {
    eng.set_phase(kPhaseMove);
    for (int b : {0, 2}) {
      const size_t mk = arena.mark();
      View T = t2(set, b);
      View c = eng.temp({no, no, nv, nv}, true);
      eng.add(c, T, 1.0, 0.0, 0);
      eng.add(T, c, 0.25, 0.0, 0);
      eng.add(T, reorder(c, {1, 0, 2, 3}), -0.25, 0.0, 1);
      eng.add(T, reorder(c, {0, 1, 3, 2}), -0.25, 0.0, 1);
      eng.add(T, reorder(c, {1, 0, 3, 2}), 0.25, 0.0, 1);
      arena.release(mk);
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
      antisymmetrize_same_spin(X);
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
  if (o->prec < 0 || o->prec > 2) { *m = "unknown precision"; return false; }
  if (o->fp_map < 0 || o->fp_map > 1) { *m = "unknown fixed-point map"; return false; }
  if (o->fp_fixed_iters < 0 || o->fp_max_iter < 1) { *m = "bad pass counts"; return false; }
  if (!(o->fp_tol > 0.0)) { *m = "fp_tol must be positive"; return false; }
  if (o->max_steps < 1) { *m = "max_steps must be >= 1"; return false; }
  if (o->tune < 0 || o->tune > 1) { *m = "tune must be 0 or 1"; return false; }
  if (o->fp_anderson < 0 || o->fp_anderson > 8) { *m = "fp_anderson must be in 0..8"; return false; }
  return true;
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

// Plan init + one residual without touching a device: the workspace peak and the
// residual's flop counts (total and by phase).
static rteom_status dry_plan(int32_t n_orb, int32_t n_occ_a, int32_t n_occ_b, int32_t n_chol,
                             int32_t core_orb, int32_t core_spin, const rteom_options& o, size_t* bytes,
                             double* flops, double* phase_flops) {
  std::unique_ptr<rteom_ctx> ctx(new rteom_ctx());
  Context& c = ctx->c;
  c.dry = true;
  c.opt = o;
  c.n = n_orb; c.nq = n_chol; c.na = n_occ_a; c.nb = n_occ_b; c.core_orb = core_orb; c.core_spin = core_spin;
  c.arena.init(nullptr, ~static_cast<size_t>(0) >> 2);
  const rteom_status st = guarded(ctx.get(), [&] {
    c.init(nullptr, nullptr);
    c.residual(c.X, c.R);
    c.antisymmetrize_same_spin(c.X);   // its temporary, for rteom_ground_state
  });
  if (st != RTEOM_OK) { g_last_error = c.err; return st; }
  *bytes = c.arena.peak() + (1 << 20);
  if (flops) *flops = c.res_flops;
  if (phase_flops)
    for (int k = 0; k < rteom::kNumPhases; ++k) phase_flops[k] = c.res_phase_flops[k];
  return RTEOM_OK;
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
  return dry_plan(n_orb, n_occ_a, n_occ_b, n_chol, core_orb, core_spin, o, bytes, nullptr, nullptr);
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
  size_t need = 0;
  double plan_flops = 0.0, plan_phase_flops[rteom::kNumPhases] = {0};
  st = dry_plan(n_orb, n_occ_a, n_occ_b, n_chol, core_orb, core_spin, o, &need, &plan_flops, plan_phase_flops);
  if (st != RTEOM_OK) return st;
  std::unique_ptr<rteom_ctx> ctx(new rteom_ctx());
  Context& c = ctx->c;
  c.opt = o;
  c.res_flops = plan_flops;       // known from the plan before the first evaluation
  for (int k = 0; k < rteom::kNumPhases; ++k) c.res_phase_flops[k] = plan_phase_flops[k];
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
constexpr uint32_t kImageVersion = 1;
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

rteom_status rteom_spectral(rteom_ctx* ctx, double e_corr, double eta, int64_t n_w, const double* omega,
                            double* a_out, double* qp_out) {
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  Context& c = ctx->c;
  if (c.core_orb < 0) { c.err = "the context has no core hole"; return RTEOM_ERR_ARG; }
  if (!omega || !a_out || n_w < 1) { c.err = "omega and a_out are required, n_w >= 1"; return RTEOM_ERR_ARG; }
  if (!std::isfinite(e_corr) || !std::isfinite(eta) || eta < 0.0) {
    c.err = "e_corr must be finite and eta finite and >= 0";
    return RTEOM_ERR_ARG;
  }
  for (int64_t j = 0; j < n_w; ++j)
    if (!std::isfinite(omega[j])) { c.err = "non-finite frequency"; return RTEOM_ERR_ARG; }
  return guarded(ctx, [&] {
    const int64_t n = c.nsteps + 1;
    // post-processing buffers: times, frequencies, weighted G, A, peak
    const size_t bytes = sizeof(double) * (size_t)(n + n_w + 2 * n + n_w + 2);
    std::unique_ptr<double, std::function<void(double*)>> buf(
        static_cast<double*>(c.be->alloc(bytes)), [&c](double* p) { if (p) c.be->release(p); });
    if (!buf) throw Error(RTEOM_ERR_OOM, "device allocation for the spectrum failed");
    double *t = buf.get(), *w = t + n, *wg = w + n_w, *a = wg + 2 * n, *qp = a + n_w;
    c.be->h2d(t, c.times.data(), sizeof(double) * n);
    c.be->h2d(w, omega, sizeof(double) * n_w);
    c.be->spectral(c.c_hist, t, n, c.eps_core + e_corr, eta, w, n_w, wg, a, qp);
    c.be->d2h(a_out, a, sizeof(double) * n_w);
    if (qp_out) c.be->d2h(qp_out, qp, sizeof(double) * 2);
  });
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
    std::vector<double> buf;
    to_planar(c, t1, t2, buf);
    for (double v : buf)
      if (!std::isfinite(v)) throw Error(RTEOM_ERR_NONFINITE, "non-finite amplitude");
    c.be->h2d(c.X, buf.data(), buf.size() * sizeof(double));
    for (int s = 0; s < 2; ++s) {
      const double* sc[2] = {c.mo[s], c.mv[s]};
      c.eng.scale(c.t1(c.X, s), sc);
    }
    const int sp[3][2] = {{0, 0}, {0, 1}, {1, 1}};
    for (int b = 0; b < 3; ++b) {
      const double* sc[4] = {c.mo[sp[b][0]], c.mo[sp[b][1]], c.mv[sp[b][0]], c.mv[sp[b][1]]};
      c.eng.scale(c.t2(c.X, b), sc);
    }
    c.energy(c.X, c.e_hist + 2 * c.nsteps);   // E(T_n) for the next trapezoid
    c.be->fill(c.dbad, 1, 0.0);
    c.failed = false;
  });
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
  *flops = cctx->c.res_flops;
  return RTEOM_OK;
}

rteom_status rteom_profile(rteom_ctx* ctx, uint32_t phase_mask) {
  if (!ctx) { g_last_error = "NULL context"; return RTEOM_ERR_ARG; }
  ctx->c.be->set_profile(phase_mask);
  return RTEOM_OK;
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
    if (flops) *flops = c.res_phase_flops[phase];
  });
}

struct rteom_batch {
  std::vector<rteom_ctx*> ctxs;
  void* exec = nullptr;
  double dt = 0.0;
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
    if (!b->exec || b->dt != dt) {
      std::vector<void*> graphs;
      for (rteom_ctx* x : b->ctxs) {
        void* e = x->c.graph_for(dt);
        if (!e) throw Error(RTEOM_ERR_STATE, "graph capture unavailable (null stream?)");
        graphs.push_back(x->c.be->captured_graph(e));
        x->c.be->sync();
      }
      if (b->exec) lead->c.be->destroy_graph(b->exec);
      b->exec = lead->c.be->combine_graphs(graphs.data(), (int)graphs.size());
      if (!b->exec) throw Error(RTEOM_ERR_HIP, "could not build the batch graph");
      b->dt = dt;
    }
    for (int32_t k = 0; k < n_steps; ++k) {
      lead->c.be->launch_graph(b->exec);
      for (rteom_ctx* x : b->ctxs) {
        ++x->c.nsteps;
        x->c.times.push_back(x->c.times.back() + dt);
      }
    }
    lead->c.be->sync();
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
  if (b->exec && !b->ctxs.empty()) b->ctxs[0]->c.be->destroy_graph(b->exec);
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
