// Host implementation of the backend operations.
//
// TEST BUILD ONLY: compiled into a separate library (librteom_hostcheck.so) so
// that the engine's host logic -- the contraction planner, the spin-blocked
// residual sequence and the step bookkeeping -- can be checked on a machine
// without a GPU.  The product library links backend_hip.hip instead and never
// contains this file.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "backend.h"

namespace rteom {

namespace {

inline int64_t off(const int64_t* idx, const int64_t* str, int nd) {
  int64_t o = 0;
  for (int d = 0; d < nd; ++d) o += idx[d] * str[d];
  return o;
}

class HostBackend : public Backend {
 public:
  void* alloc(size_t bytes) override { return std::calloc(1, bytes); }
  void release(void* p) override { std::free(p); }
  void h2d(void* d, const void* s, size_t b) override { std::memcpy(d, s, b); }
  void d2h(void* d, const void* s, size_t b) override { std::memcpy(d, s, b); }
  void d2d(void* d, const void* s, size_t b) override { std::memmove(d, s, b); }
  void fill(double* p, int64_t n, double v) override { std::fill(p, p + n, v); }
  void sync() override {}
  bool ok(std::string*) override { return true; }
  int64_t energy_partials() const override { return 4096; }

  void gemm(const GemmOp& g) override {
    const bool ac = g.a_im != nullptr, bc = g.b_im != nullptr;
    const bool cc = ac || bc;
    for (int64_t b = 0; b < g.batch; ++b)
      for (int64_t m = 0; m < g.M; ++m)
        for (int64_t n = 0; n < g.N; ++n) {
          double sr = 0.0, si = 0.0;
          for (int64_t k = 0; k < g.K; ++k) {
            const int64_t ia = b * g.a_sb + m * g.a_sm + k * g.a_sk;
            const int64_t ib = b * g.b_sb + k * g.b_sk + n * g.b_sn;
            const double ar = g.a_re[ia], ai = ac ? g.a_im[ia] : 0.0;
            const double br = g.b_re[ib], bi = bc ? g.b_im[ib] : 0.0;
            sr += ar * br - ai * bi;
            si += ar * bi + ai * br;
          }
          const int64_t ic = b * g.c_sb + m * g.c_sm + n * g.c_sn;
          g.c_re[ic] = g.alpha * sr + (g.beta ? g.c_re[ic] : 0.0);
          if (cc) g.c_im[ic] = g.alpha * si + (g.beta ? g.c_im[ic] : 0.0);
        }
  }

  void permute(const PermOp& p) override {
    int64_t total = 1;
    for (int d = 0; d < p.nd; ++d) total *= p.dim[d];
    // read everything first so that in == out works for any strides
    std::vector<double> vr(total), vi(total);
    int64_t idx[kMaxDims] = {0};
    for (int64_t t = 0; t < total; ++t) {
      int64_t r = t;
      for (int d = p.nd - 1; d >= 0; --d) {
        idx[d] = r % p.dim[d];
        r /= p.dim[d];
      }
      const int64_t io = off(idx, p.in_str, p.nd);
      double xr = p.in_re[io], xi = p.in_im ? p.in_im[io] : 0.0;
      double s = 1.0;
      for (int d = 0; d < p.nd; ++d)
        if (p.scale[d]) s *= p.scale[d][idx[d]];
      vr[t] = s * (p.alpha_re * xr - p.alpha_im * xi);
      vi[t] = s * (p.alpha_re * xi + p.alpha_im * xr);
      if (p.alpha_re == 0.0 && p.alpha_im == 0.0) vr[t] = vi[t] = 0.0;
    }
    for (int64_t t = 0; t < total; ++t) {
      int64_t r = t;
      for (int d = p.nd - 1; d >= 0; --d) {
        idx[d] = r % p.dim[d];
        r /= p.dim[d];
      }
      const int64_t oo = off(idx, p.out_str, p.nd);
      p.out_re[oo] = vr[t] + (p.beta ? p.out_re[oo] : 0.0);
      if (p.out_im) p.out_im[oo] = vi[t] + (p.beta ? p.out_im[oo] : 0.0);
    }
  }

  void ss(const SsOp& op) override {
    const int64_t n1 = op.n1, n2 = op.n2, np1 = npairs(n1), np2 = npairs(n2);
    auto pidx = [](int64_t i, int64_t j, int64_t n) { return pair_start(i, n) + j - i - 1; };
    const bool cx = op.y_im != nullptr || op.x_im != nullptr;
    auto X = [&](int pl, int64_t o) { return pl ? op.x_im[o] : op.x_re[o]; };
    double* Y[2] = {op.y_re, op.y_im};
    double* Xw[2] = {op.x_re, op.x_im};
    const int npl = cx ? 2 : 1;
    switch (op.mode) {
      case SsOp::kExpand:
        for (int64_t ii = 0; ii < op.ci; ++ii)
          for (int64_t jj = 0; jj < op.cj; ++jj)
            for (int64_t a = 0; a < n2; ++a)
              for (int64_t b = 0; b < n2; ++b) {
                const int64_t i = op.i0 + ii, j = op.j0 + jj, xo = ((ii * op.cj + jj) * n2 + a) * n2 + b;
                for (int pl = 0; pl < npl; ++pl) {
                  double v = 0.0;
                  if (i != j && a != b) {
                    const double sg = (i < j ? 1.0 : -1.0) * (a < b ? 1.0 : -1.0);
                    v = op.alpha * sg * Y[pl][pidx(std::min(i, j), std::max(i, j), n1) * np2 +
                                              pidx(std::min(a, b), std::max(a, b), n2)];
                  }
                  Xw[pl][xo] = v + (op.beta ? Xw[pl][xo] : 0.0);
                }
              }
        break;
      case SsOp::kAccum: {
        // the definition: the block's antisymmetrised contributions, pair by pair
        auto in_i = [&](int64_t k) { return k >= op.i0 && k < op.i0 + op.ci; };
        auto in_j = [&](int64_t k) { return k >= op.j0 && k < op.j0 + op.cj; };
        auto xv = [&](int pl, int64_t i, int64_t j, int64_t a, int64_t b) {
          return X(pl, (((i - op.i0) * op.cj + (j - op.j0)) * n2 + a) * n2 + b);
        };
        for (int64_t k = 0; k < n1; ++k)
          for (int64_t l = k + 1; l < n1; ++l)
            for (int64_t a = 0; a < n2; ++a)
              for (int64_t b = a + 1; b < n2; ++b)
                for (int pl = 0; pl < npl; ++pl) {
                  double v = 0.0;
                  if (in_i(k) && in_j(l)) v += xv(pl, k, l, a, b) - (op.anti2 ? xv(pl, k, l, b, a) : 0.0);
                  if (op.anti1 && in_i(l) && in_j(k)) v -= xv(pl, l, k, a, b) - (op.anti2 ? xv(pl, l, k, b, a) : 0.0);
                  Y[pl][pidx(k, l, n1) * np2 + pidx(a, b, n2)] += op.alpha * v;
                }
        break;
      }
      case SsOp::kAccumRows:
        for (int64_t pp = 0; pp < op.ci; ++pp)
          for (int64_t a = 0; a < n2; ++a)
            for (int64_t b = a + 1; b < n2; ++b)
              for (int pl = 0; pl < npl; ++pl) {
                const double v = X(pl, (pp * n2 + a) * n2 + b) - (op.anti2 ? X(pl, (pp * n2 + b) * n2 + a) : 0.0);
                Y[pl][(op.i0 + pp) * np2 + pidx(a, b, n2)] += op.alpha * v;
              }
        break;
      case SsOp::kT1T1:
        for (int64_t p = 0; p < np1; ++p)
          for (int64_t q = 0; q < np2; ++q) {
            const int64_t i = op.pt.oi[p], j = op.pt.oj[p], a = op.pt.va[q], b = op.pt.vb[q];
            auto ur = [&](int64_t x, int64_t y) { return op.u_re[x * n2 + y]; };
            auto ui = [&](int64_t x, int64_t y) { return op.u_im[x * n2 + y]; };
            const double vr = ur(i, a) * ur(j, b) - ui(i, a) * ui(j, b) - (ur(i, b) * ur(j, a) - ui(i, b) * ui(j, a));
            const double vi = ur(i, a) * ui(j, b) + ui(i, a) * ur(j, b) - (ur(i, b) * ui(j, a) + ui(i, b) * ur(j, a));
            const int64_t o = p * np2 + q;
            op.y_re[o] = op.alpha * vr + (op.beta ? op.y_re[o] : 0.0);
            op.y_im[o] = op.alpha * vi + (op.beta ? op.y_im[o] : 0.0);
          }
        break;
      case SsOp::kMask:
        for (int64_t p = 0; p < np1; ++p)
          for (int64_t q = 0; q < np2; ++q) {
            const double m = op.m1[op.pt.oi[p]] * op.m1[op.pt.oj[p]] * op.m2[op.pt.va[q]] * op.m2[op.pt.vb[q]];
            for (int pl = 0; pl < npl; ++pl) Y[pl][p * np2 + q] *= m;
          }
        break;
      case SsOp::kPackSlab: {
        const int64_t base = pair_start(op.i0, n1);
        const int64_t rest = op.pair2 ? n2 * n2 : n2, nq = op.pair2 ? np2 : n2;
        for (int64_t ee = 0; ee < op.ci; ++ee)
          for (int64_t f = op.i0 + ee + 1; f < n1; ++f) {
            const int64_t p = pidx(op.i0 + ee, f, n1) - base;
            const int64_t xo = (ee * n1 + f) * rest;
            for (int pl = 0; pl < npl; ++pl) {
              if (op.pair2) {
                for (int64_t a = 0; a < n2; ++a)
                  for (int64_t b = a + 1; b < n2; ++b)
                    Y[pl][p * nq + pidx(a, b, n2)] = op.alpha * (X(pl, xo + a * n2 + b) - X(pl, xo + b * n2 + a));
              } else {
                for (int64_t c = 0; c < n2; ++c) Y[pl][p * nq + c] = op.alpha * X(pl, xo + c);
              }
            }
          }
        break;
      }
    }
  }

  void update(const UpdateOp& u) override {
    const int64_t n1 = u.lay.n1(), nss = u.lay.nss(), nab = u.lay.nab(), no = u.lay.no, nv = u.lay.nv;
    const int64_t npv = u.lay.npv(), total = u.lay.size();
    (void)nab;
    double dmax = 0.0;
    for (int64_t k = 0; k < total; ++k) {
      double mask, dd;
      if (k < 2 * n1) {
        const int s = (int)(k / n1);
        const int64_t r = k % n1, i = r / nv, a = r % nv;
        mask = u.sv.mo[s][i] * u.sv.mv[s][a];
        dd = u.sv.fo[s][i] - u.sv.fv[s][a];
      } else if (k < u.lay.off_ab()) {
        const int64_t k2 = k - 2 * n1;
        const int s = (int)(k2 / nss);
        const int64_t r = k2 % nss, p = r / npv, q = r % npv;
        const int64_t i = u.pt.oi[p], j = u.pt.oj[p], a = u.pt.va[q], b = u.pt.vb[q];
        mask = u.sv.mo[s][i] * u.sv.mo[s][j] * u.sv.mv[s][a] * u.sv.mv[s][b];
        dd = u.sv.fo[s][i] + u.sv.fo[s][j] - u.sv.fv[s][a] - u.sv.fv[s][b];
      } else {
        int64_t r = k - u.lay.off_ab();
        const int64_t b = r % nv; r /= nv;
        const int64_t a = r % nv; r /= nv;
        const int64_t j = r % no, i = r / no;
        mask = u.sv.mo[0][i] * u.sv.mo[1][j] * u.sv.mv[0][a] * u.sv.mv[1][b];
        dd = u.sv.fo[0][i] + u.sv.fo[1][j] - u.sv.fv[0][a] - u.sv.fv[1][b];
      }
      const double xr = u.x_re[k], xi = u.x_im[k], rr = u.r_re[k], ri = u.r_im[k];
      if (u.mode == 2) {   // Jacobi step towards R(T) = 0
        double nr = dd != 0.0 ? xr + rr / dd : 0.0, ni = dd != 0.0 ? xi + ri / dd : 0.0;
        if (mask == 0.0) nr = ni = 0.0;
        const double dr = nr - xr, di = ni - xi;
        dmax = std::max(dmax, std::sqrt(dr * dr + di * di));
        if (std::isnan(nr) || std::isnan(ni)) dmax = NAN;
        u.x_re[k] = nr;
        u.x_im[k] = ni;
        continue;
      }
      double hr, hi;  // rhs
      if (u.start) {
        hr = xr - u.h * ri;
        hi = xi + u.h * rr;
        if (u.rhs_re) {
          u.rhs_re[k] = hr;
          u.rhs_im[k] = hi;
        }
      } else {
        hr = u.rhs_re[k];
        hi = u.rhs_im[k];
      }
      double nr, ni;
      if (u.mode == 0) {
        nr = hr - u.h * ri;
        ni = hi + u.h * rr;
      } else {
        // (rhs + i h (r + D x)) / (1 + i h D)
        const double pr = rr + dd * xr, pi = ri + dd * xi;
        const double numr = hr - u.h * pi, numi = hi + u.h * pr;
        const double den_r = 1.0, den_i = u.h * dd, den2 = den_r * den_r + den_i * den_i;
        nr = (numr * den_r + numi * den_i) / den2;
        ni = (numi * den_r - numr * den_i) / den2;
      }
      if (mask == 0.0) nr = ni = 0.0;
      const double dr = nr - xr, di = ni - xi;
      dmax = std::max(dmax, std::sqrt(dr * dr + di * di));
      if (std::isnan(nr) || std::isnan(ni)) dmax = NAN;
      u.x_re[k] = nr;
      u.x_im[k] = ni;
    }
    if (std::isnan(dmax) || dmax > *u.delta || std::isnan(*u.delta)) *u.delta = dmax;
  }

  void energy(const EnergyOp& e) override {
    const int64_t no = e.lay.no, nv = e.lay.nv, n1 = e.lay.n1(), npv = e.lay.npv();
    auto pidx = [](int64_t i, int64_t j, int64_t n) { return pair_start(i, n) + j - i - 1; };
    const double* xr = e.x_re;
    const double* xi = e.x_im;
    auto t1r = [&](int s, int64_t i, int64_t a) { return xr[s * n1 + i * nv + a]; };
    auto t1i = [&](int s, int64_t i, int64_t a) { return xi[s * n1 + i * nv + a]; };
    double er = 0.0, ei = 0.0;
    if (e.include_ft1)
      for (int s = 0; s < 2; ++s)
        for (int64_t i = 0; i < no; ++i)
          for (int64_t a = 0; a < nv; ++a) {
            const double fv = e.fov[s][i * e.fov_ld + a];
            er += fv * t1r(s, i, a);
            ei += fv * t1i(s, i, a);
          }
    for (int64_t i = 0; i < no; ++i)
      for (int64_t a = 0; a < nv; ++a)
        for (int64_t j = 0; j < no; ++j)
          for (int64_t b = 0; b < nv; ++b) {
            const double J = e.jov[((i * nv + a) * no + j) * nv + b];
            const int64_t p = e.lay.off_ab() + ((i * no + j) * nv + a) * nv + b;
            double wr = xr[p], wi = xi[p];
            // 1/2 (T_aa + T_bb) + T_ab, the same-spin elements from pair storage
            if (i != j && a != b) {
              const double sg = 0.5 * (i < j ? 1.0 : -1.0) * (a < b ? 1.0 : -1.0);
              const int64_t q = pidx(std::min(i, j), std::max(i, j), no) * npv + pidx(std::min(a, b), std::max(a, b), nv);
              wr += sg * (xr[e.lay.off_ss(0) + q] + xr[e.lay.off_ss(1) + q]);
              wi += sg * (xi[e.lay.off_ss(0) + q] + xi[e.lay.off_ss(1) + q]);
            }
            for (int s = 0; s < 2; ++s) {
              // 1/2 t_ia t_jb - 1/2 t_ib t_ja (same spin)
              double ar = t1r(s, i, a), ai = t1i(s, i, a), br = t1r(s, j, b), bi = t1i(s, j, b);
              wr += 0.5 * (ar * br - ai * bi);
              wi += 0.5 * (ar * bi + ai * br);
              ar = t1r(s, i, b); ai = t1i(s, i, b); br = t1r(s, j, a); bi = t1i(s, j, a);
              wr -= 0.5 * (ar * br - ai * bi);
              wi -= 0.5 * (ar * bi + ai * br);
            }
            {
              const double ar = t1r(0, i, a), ai = t1i(0, i, a), br = t1r(1, j, b), bi = t1i(1, j, b);
              wr += ar * br - ai * bi;
              wi += ar * bi + ai * br;
            }
            er += J * wr;
            ei += J * wi;
          }
    e.e_out[0] = er;
    e.e_out[1] = ei;
  }

  void dot(const double* a, const double* b, int64_t n, double*, double* out) override {
    double acc = 0.0;
    for (int64_t k = 0; k < n; ++k) acc += a[k] * b[k];
    *out = acc;
  }

  void spectral(const double* c, const double* t, int64_t n, double shift, double eta, const double* omega,
                int64_t n_w, double* wg, double* a, double* qp) override {
    if (n < 1 || n_w < 1) return;
    for (int64_t k = 0; k < n; ++k) {
      const double w = n > 1 ? 0.5 * ((k + 1 < n ? t[k + 1] : t[k]) - (k > 0 ? t[k - 1] : t[k])) : 0.0;
      const double mag = std::exp(c[2 * k]) * w, ph = c[2 * k + 1] - shift * t[k];
      wg[2 * k] = mag * std::sin(ph);
      wg[2 * k + 1] = -mag * std::cos(ph);
    }
    int64_t best = 0;
    for (int64_t j = 0; j < n_w; ++j) {
      double im = 0.0;
      for (int64_t k = 0; k < n; ++k)
        im += std::exp(-eta * t[k]) * (wg[2 * k] * std::sin(omega[j] * t[k]) + wg[2 * k + 1] * std::cos(omega[j] * t[k]));
      a[j] = -im / M_PI;
      if (a[j] > a[best]) best = j;
    }
    double pos = omega[best];
    if (best > 0 && best + 1 < n_w) {
      const double y0 = a[best - 1], y1 = a[best], y2 = a[best + 1], den = y0 - 2.0 * y1 + y2;
      pos = omega[best] + (den != 0.0 ? 0.5 * (y0 - y2) / den : 0.0) * (omega[1] - omega[0]);
    }
    qp[0] = pos;
    qp[1] = a[best];
  }

  void spectral_peaks(const double* a, const double* omega, int64_t n_w, int k, double* out) override {
    std::vector<int64_t> taken;
    for (int r = 0; r < k; ++r) {
      int64_t bi = -1;
      for (int64_t j = 1; j + 1 < n_w; ++j) {
        if (!(a[j] > a[j - 1] && a[j] >= a[j + 1])) continue;
        if (std::find(taken.begin(), taken.end(), j) != taken.end()) continue;
        if (bi < 0 || a[j] > a[bi]) bi = j;
      }
      if (bi < 0) break;
      const double y0 = a[bi - 1], y1 = a[bi], y2 = a[bi + 1], den = y0 - 2.0 * y1 + y2;
      out[2 * taken.size()] = omega[bi] + (den != 0.0 ? 0.5 * (y0 - y2) / den : 0.0) * (omega[1] - omega[0]);
      out[2 * taken.size() + 1] = a[bi];
      taken.push_back(bi);
    }
    out[2 * k] = (double)taken.size();
  }

  void cumulant_append(double* c, double* e, const double* en, int64_t* step, double h, double* bad) override {
    // C + i h (E_k + E_{k+1})
    const int64_t k = *step;
    const double sr = e[2 * k] + en[0], si = e[2 * k + 1] + en[1];
    c[2 * (k + 1)] = c[2 * k] - h * si;
    c[2 * (k + 1) + 1] = c[2 * k + 1] + h * sr;
    e[2 * (k + 1)] = en[0];
    e[2 * (k + 1) + 1] = en[1];
    *step = k + 1;
    if (!std::isfinite(en[0]) || !std::isfinite(en[1]) || !std::isfinite(c[2 * (k + 1)]) ||
        !std::isfinite(c[2 * (k + 1) + 1]))
      *bad = 1.0;
  }
};

}  // namespace

Backend* make_host_backend() { return new HostBackend(); }

}  // namespace rteom
