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

  void pairs(const PairOp& op) override {
    const int64_t n1 = op.n1, n2 = op.n2;
    const int64_t rest = op.pair2 ? n2 * n2 : n2;
    const int64_t nq = op.pair2 ? n2 * (n2 - 1) / 2 : n2;
    auto pidx = [](int64_t i, int64_t j, int64_t n) { return i * (2 * n - i - 1) / 2 + (j - i - 1); };
    for (int64_t blk = 0; blk < op.nblk; ++blk)
      for (int64_t i = 0; i < n1; ++i)
        for (int64_t j = 0; j < n1; ++j)
          for (int64_t c = 0; c < rest; ++c) {
            const int64_t a = op.pair2 ? c / n2 : 0, b = op.pair2 ? c % n2 : c;
            const int64_t xo = blk * op.x_bs + (i * n1 + j) * rest + c;
            if (op.mode == 0) {
              if (i >= j || (op.pair2 && a >= b)) continue;
              const int64_t yo = blk * op.y_bs + pidx(i, j, n1) * nq + (op.pair2 ? pidx(a, b, n2) : b);
              const int64_t xs = blk * op.x_bs + (j * n1 + i) * rest + c;
              op.y_re[yo] = op.alpha * (op.x_re[xo] - (op.anti ? op.x_re[xs] : 0.0));
              if (op.y_im) op.y_im[yo] = op.alpha * (op.x_im[xo] - (op.anti ? op.x_im[xs] : 0.0));
            } else {
              double vr = 0.0, vi = 0.0;
              if (i != j && (!op.pair2 || a != b)) {
                double sg = i < j ? 1.0 : -1.0;
                int64_t q = b;
                if (op.pair2) {
                  q = pidx(std::min(a, b), std::max(a, b), n2);
                  if (b < a) sg = -sg;
                }
                const int64_t yo = blk * op.y_bs + pidx(std::min(i, j), std::max(i, j), n1) * nq + q;
                vr = op.alpha * sg * op.y_re[yo];
                if (op.y_im) vi = op.alpha * sg * op.y_im[yo];
              }
              op.x_re[xo] = vr + (op.beta ? op.x_re[xo] : 0.0);
              if (op.x_im) op.x_im[xo] = vi + (op.beta ? op.x_im[xo] : 0.0);
            }
          }
  }

  void update(const UpdateOp& u) override {
    const int64_t n1 = u.lay.n1(), n2 = u.lay.n2(), no = u.lay.no, nv = u.lay.nv;
    const int64_t total = u.lay.size();
    double dmax = 0.0;
    for (int64_t k = 0; k < total; ++k) {
      double mask, dd;
      if (k < 2 * n1) {
        const int s = (int)(k / n1);
        const int64_t r = k % n1, i = r / nv, a = r % nv;
        mask = u.sv.mo[s][i] * u.sv.mv[s][a];
        dd = u.sv.fo[s][i] - u.sv.fv[s][a];
      } else {
        const int64_t k2 = k - 2 * n1;
        const int blk = (int)(k2 / n2);
        const int s1 = blk == 2 ? 1 : 0, s2 = blk == 0 ? 0 : 1;
        int64_t r = k2 % n2;
        const int64_t b = r % nv; r /= nv;
        const int64_t a = r % nv; r /= nv;
        const int64_t j = r % no, i = r / no;
        mask = u.sv.mo[s1][i] * u.sv.mo[s2][j] * u.sv.mv[s1][a] * u.sv.mv[s2][b];
        dd = u.sv.fo[s1][i] + u.sv.fo[s2][j] - u.sv.fv[s1][a] - u.sv.fv[s2][b];
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
        u.rhs_re[k] = hr;
        u.rhs_im[k] = hi;
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
    const int64_t no = e.lay.no, nv = e.lay.nv, n1 = e.lay.n1(), n2 = e.lay.n2();
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
            const int64_t p = ((i * no + j) * nv + a) * nv + b;
            double wr = 0.0, wi = 0.0;
            // 1/2 (T_aa + T_bb) + T_ab
            wr += 0.5 * (xr[2 * n1 + p] + xr[2 * n1 + 2 * n2 + p]) + xr[2 * n1 + n2 + p];
            wi += 0.5 * (xi[2 * n1 + p] + xi[2 * n1 + 2 * n2 + p]) + xi[2 * n1 + n2 + p];
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
