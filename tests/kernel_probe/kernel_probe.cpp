// Kernel probe (test program, GPU): the GEMM backend on every operand layout,
// complex combination, ragged size, split-K, broadcast batch and tile shape
// (forced), against host loops; tile shapes and the converted-operand paths must
// agree bitwise.  Also the permute kernels and the same-spin pair operations against
// host loops.
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <vector>
#include <string>
#include <chrono>
#include <algorithm>
#include "../../paper_2301_04249_amd/csrc/backend.h"
using namespace rteom;

static int check(Backend* be) {
  int shapes[][5] = {{1,1,1,1,1},{16,16,4,1,1},{64,64,16,1,1},{65,70,17,1,1},{130,33,100,3,1},{7,200,9,2,1},
                     {8,111,3000,1,5},{20,9,1000,1,64},{65,70,17,1,2},{64,64,160,1,3},
                     {600,1000,40,1,1},{1000,600,40,2,1},{577,130,36,1,1},{300,260,70,1,3}};
  int fails = 0, runs = 0;
  srand(1);
  for (int prec = 0; prec < 4; ++prec)
  for (auto& sh : shapes) {
    long M = sh[0], N = sh[1], K = sh[2], B = sh[3]; int S = sh[4];
    for (int bcast = 0; bcast < (B > 1 ? 2 : 1); ++bcast)
    for (int lay = 0; lay < 4; ++lay) for (int cx = 0; cx < 4; ++cx) {
      bool akc = lay & 1, bkc = lay & 2, ac = cx & 1, bc = cx & 2;
      long na = B*M*K, nb = B*K*N, nc = B*M*N;
      std::vector<double> A(2*na), Bv(2*nb), C(2*nc), Cref(2*nc), Cout(2*nc), C0(2*nc), C1(2*nc);
      for (auto& x : A) x = rand()/(double)RAND_MAX - 0.5;
      for (auto& x : Bv) x = rand()/(double)RAND_MAX - 0.5;
      for (auto& x : C) x = rand()/(double)RAND_MAX - 0.5;
      GemmOp g;
      std::vector<double> Cabs(nc); g.M=M; g.N=N; g.K=K; g.batch=B;
      g.a_sm = akc ? K : 1; g.a_sk = akc ? 1 : M; g.a_sb = bcast ? 0 : M*K;   // bcast: one A for every batch entry
      g.b_sk = bkc ? 1 : N; g.b_sn = bkc ? K : 1; g.b_sb = K*N;
      g.c_sm = N; g.c_sn = 1; g.c_sb = M*N; g.alpha = 0.75; g.beta = 1; g.prec = prec;
      double* dP = nullptr;
      if (S > 1) { dP = (double*)be->alloc(16L*S*M*N); g.splitk = S; g.partial = dP; }
      if (prec == 3) {
        // rows of A and columns of B over 2^-20 .. 2^20 (the per-row scaling's case);
        // checked element by element against the sum of magnitudes
        for (long b=0;b<(bcast?1:B);++b) for (long m=0;m<M;++m) for (long k=0;k<K;++k) {
          long ia = b*M*K + m*g.a_sm + k*g.a_sk;
          A[ia] = std::ldexp(A[ia], (int)(m % 41) - 20); A[na+ia] = std::ldexp(A[na+ia], (int)(m % 41) - 20);
        }
        for (long b=0;b<B;++b) for (long n=0;n<N;++n) for (long k=0;k<K;++k) {
          long ib = b*g.b_sb + k*g.b_sk + n*g.b_sn;
          Bv[ib] = std::ldexp(Bv[ib], (int)(n % 37) - 18); Bv[nb+ib] = std::ldexp(Bv[nb+ib], (int)(n % 37) - 18);
        }
      }
      for (long b=0;b<B;++b) for (long m=0;m<M;++m) for (long n=0;n<N;++n) {
        double sr=0, si=0, sa=0;
        for (long k=0;k<K;++k) {
          long ia = b*g.a_sb + m*g.a_sm + k*g.a_sk, ib = b*g.b_sb + k*g.b_sk + n*g.b_sn;
          double ar=A[ia], ai= ac? A[na+ia]:0, br=Bv[ib], bi = bc? Bv[nb+ib]:0;
          sr += ar*br - ai*bi; si += ar*bi + ai*br;
          sa += (std::fabs(ar) + std::fabs(ai)) * (std::fabs(br) + std::fabs(bi));
        }
        long ic = b*g.c_sb + m*g.c_sm + n*g.c_sn;
        Cref[ic] = 0.75*sr + C[ic]; Cref[nc+ic] = 0.75*si + C[nc+ic];
        Cabs[ic] = 0.75*sa + std::fabs(C[ic]) + std::fabs(C[nc+ic]);
      }
      double *dA=(double*)be->alloc(16*na), *dB=(double*)be->alloc(16*nb), *dC=(double*)be->alloc(16*nc);
      be->h2d(dA, A.data(), 16*na); be->h2d(dB, Bv.data(), 16*nb);
      g.a_re=dA; g.a_im = ac? dA+na : nullptr; g.b_re=dB; g.b_im = bc? dB+nb : nullptr;
      g.c_re=dC; g.c_im = (ac||bc) ? dC+nc : nullptr;
      double* dS = nullptr;
      if (prec >= 1) dS = (double*)be->alloc(8 * split_doubles(M, N, K, bcast ? 1 : B, B, ac, bc, prec));
      for (int vv = prec == 3 ? 4 : -1; vv < (prec >= 1 ? 9 : 6); ++vv) {
        // prec 0: -1..5; prec 1, 2: -1..3 converted while staging, then -1..3 converted
        // before; prec 3 (converted before only): -1..3
        const int v = (prec >= 1 && vv >= 4) ? vv - 5 : vv;
        g.split = (prec >= 1 && vv >= 4) ? dS : nullptr;
        be->force_tile(v);
        be->h2d(dC, C.data(), 16*nc);
        be->gemm(g); be->sync();
        be->d2h(Cout.data(), dC, 16*nc);
        double e=0, mx=1; long nn = (ac||bc) ? 2*nc : nc;
        for (long i=0;i<nn;++i) { e = std::fmax(e, std::fabs(Cout[i]-Cref[i])); mx = std::fmax(mx, std::fabs(Cref[i])); }
        e /= mx;
        if (prec == 3) {
          e = 0;
          for (long i=0;i<nn;++i) e = std::fmax(e, std::fabs(Cout[i]-Cref[i]) / Cabs[i % nc]);
        }
        std::string m; bool ok = be->ok(&m);
        ++runs;
        const double tol = prec == 0 ? 1e-12 : (prec == 1 ? 2e-5 : (prec == 2 ? 2e-3 : 1e-5));
        // every tile shape of one kernel family gives bitwise the same result; bf16x3
        // on converted operands runs the 32x32x16 matrix cores (another k grouping
        // than the converting 16x16x32 kernel), so it has a reference of its own
        bool same = true;
        const bool own = prec >= 2 && vv >= 4;
        if (vv == 0) C0 = Cout;
        if (own && vv == 4) C1 = Cout;
        else if (vv > 0 && v >= 0) same = std::memcmp((own ? C1 : C0).data(), Cout.data(), sizeof(double) * nn) == 0;
        if (prec > 0 && K <= 16) continue;   // short sums run in float64 on the vector units
        if (e > tol || !ok || !same) {
          ++fails;
          printf("FAIL p=%d v=%d split=%d S=%d M=%ld N=%ld K=%ld B=%ld akc=%d bkc=%d ac=%d bc=%d err=%.3e same=%d %s\n",
                 prec, v, (int)(g.split != nullptr), S, M, N, K, B, akc, bkc, ac, bc, e, (int)same, m.c_str());
        }
      }
      g.split = nullptr;
      if (dS) be->release(dS);
      be->force_tile(-1);
      be->release(dA); be->release(dB); be->release(dC); if (dP) be->release(dP);
    }
  }
  printf("gemm probe: %d runs, %d failures\n", runs, fails);
  fflush(stdout);
  return fails;
}

// Permute check: 4-d index orders, real and complex input and output, with and
// without beta, against host loops.
static int check_permute(Backend* be) {
  int fails = 0, runs = 0;
  srand(7);
  const int shapes[][4] = {{5, 7, 33, 40}, {64, 3, 17, 96}, {1, 9, 70, 33}, {12, 12, 12, 12}};
  const int perms[][4] = {{0, 1, 2, 3}, {0, 1, 3, 2}, {3, 2, 1, 0}, {2, 0, 3, 1}, {1, 3, 0, 2}};
  for (auto& sh : shapes)
    for (auto& pm : perms)
      for (int cx = 0; cx < 4; ++cx) {
        const bool cin = cx & 1, cout_ = (cx & 2) || cin, beta = cx == 3;
        int64_t n = 1;
        for (int d = 0; d < 4; ++d) n *= sh[d];
        // input strides: row-major over dims in order; output row-major over dims permuted by pm
        int64_t istr[4], ostr[4], acc = 1;
        for (int d = 3; d >= 0; --d) { istr[d] = acc; acc *= sh[d]; }
        acc = 1;
        for (int q = 3; q >= 0; --q) { ostr[pm[q]] = acc; acc *= sh[pm[q]]; }
        std::vector<double> in(2 * n), out(2 * n), ref(2 * n), res(2 * n), sc(sh[1]);
        for (auto& x : in) x = rand() / (double)RAND_MAX - 0.5;
        for (auto& x : out) x = rand() / (double)RAND_MAX - 0.5;
        for (auto& x : sc) x = rand() / (double)RAND_MAX + 0.5;
        const double ar = 0.7, ai = cout_ ? -0.3 : 0.0;
        ref = out;
        for (int64_t i0 = 0; i0 < sh[0]; ++i0) for (int64_t i1 = 0; i1 < sh[1]; ++i1)
        for (int64_t i2 = 0; i2 < sh[2]; ++i2) for (int64_t i3 = 0; i3 < sh[3]; ++i3) {
          const int64_t io = i0 * istr[0] + i1 * istr[1] + i2 * istr[2] + i3 * istr[3];
          const int64_t oo = i0 * ostr[0] + i1 * ostr[1] + i2 * ostr[2] + i3 * ostr[3];
          const double xr = in[io], xi = cin ? in[n + io] : 0.0, s = sc[i1];
          double vr = s * (ar * xr - ai * xi), vi = s * (ar * xi + ai * xr);
          if (beta) { vr += out[oo]; vi += out[n + oo]; }
          ref[oo] = vr;
          if (cout_) ref[n + oo] = vi;
        }
        double *dI = (double*)be->alloc(16 * n), *dO = (double*)be->alloc(16 * n), *dS = (double*)be->alloc(8 * sh[1]);
        be->h2d(dI, in.data(), 16 * n); be->h2d(dO, out.data(), 16 * n); be->h2d(dS, sc.data(), 8 * sh[1]);
        PermOp p; p.nd = 4;
        for (int d = 0; d < 4; ++d) { p.dim[d] = sh[d]; p.in_str[d] = istr[d]; p.out_str[d] = ostr[d]; }
        p.scale[1] = dS;
        p.in_re = dI; p.in_im = cin ? dI + n : nullptr; p.out_re = dO; p.out_im = cout_ ? dO + n : nullptr;
        p.alpha_re = ar; p.alpha_im = ai; p.beta = beta;
        be->permute(p); be->sync();
        be->d2h(res.data(), dO, 16 * n);
        const int64_t nn = cout_ ? 2 * n : n;
        double e = 0, mx = 1e-300;
        for (int64_t i = 0; i < nn; ++i) { e = std::fmax(e, std::fabs(res[i] - ref[i])); mx = std::fmax(mx, std::fabs(ref[i])); }
        bool ok = e <= 1e-14 * mx;   // device code may contract a*b - c*d into an fma
        std::string m;
        ok = ok && be->ok(&m);
        ++runs;
        if (!ok) { ++fails; printf("PERMUTE FAIL shape %d %d %d %d perm %d %d %d %d cx %d %s\n", sh[0], sh[1], sh[2], sh[3], pm[0], pm[1], pm[2], pm[3], cx, m.c_str()); }
        be->release(dI); be->release(dO); be->release(dS);
      }
  printf("permute probe: %d runs, %d failures\n", runs, fails);
  return fails;
}

// Same-spin pair operations (SsOp) against host loops written from their definitions:
// pairs i < j in lexicographic order, sign -1 per swapped pair, every mode and flag,
// blocks of rows and columns that do and do not overlap, real and complex data.
static int check_pairs(Backend* be) {
  int fails = 0, runs = 0;
  srand(11);
  auto pidx = [](int64_t i, int64_t j, int64_t n) {   // position of (i < j) among the pairs of n
    int64_t p = 0;
    for (int64_t a = 0; a < i; ++a) p += n - 1 - a;
    return p + (j - i - 1);
  };
  const int64_t dims[][2] = {{2, 3}, {5, 4}, {7, 17}, {9, 40}};
  // blocks (i0, ci, j0, cj) as fractions of n1: whole, rows, columns, overlapping, disjoint
  for (auto& d : dims)
    for (int mode = 0; mode <= 5; ++mode)
      for (int variant = 0; variant < 16; ++variant) {
        const int64_t n1 = d[0], n2 = d[1], np1 = n1 * (n1 - 1) / 2, np2 = n2 * (n2 - 1) / 2;
        const bool cx = variant & 1;
        const int anti1 = (variant >> 1) & 1, anti2 = (variant >> 2) & 1, beta = (variant >> 3) & 1;
        int64_t i0 = 0, ci = n1, j0 = 0, cj = n1;
        const int blk = variant % 5;
        if (blk == 1) { i0 = n1 / 3; ci = n1 - n1 / 3 - (n1 > 2 ? 1 : 0); }
        if (blk == 2) { j0 = n1 / 2; cj = n1 - n1 / 2; }
        if (blk == 3) { i0 = 0; ci = (n1 + 1) / 2; j0 = n1 / 3; cj = n1 - n1 / 3; }
        if (blk == 4) { i0 = n1 / 2; ci = n1 - n1 / 2; j0 = 0; cj = n1 / 2 > 0 ? n1 / 2 : 1; }
        SsOp op;
        op.mode = mode; op.n1 = n1; op.n2 = n2; op.anti1 = anti1; op.anti2 = anti2; op.beta = beta;
        op.alpha = 0.625;
        int64_t nx = 0, ny = np1 * np2;
        if (mode == SsOp::kExpand || mode == SsOp::kAccum) { op.i0 = i0; op.ci = ci; op.j0 = j0; op.cj = cj; nx = ci * cj * n2 * n2; }
        if (mode == SsOp::kAccumRows) { op.i0 = np1 / 4; op.ci = np1 - np1 / 4; nx = op.ci * n2 * n2; }
        if (mode == SsOp::kT1T1) nx = n1 * n2;   // the t1 operand
        if (mode == SsOp::kMask) nx = n1 + n2;   // the two mask vectors
        int64_t pack_rows = 0;
        if (mode == SsOp::kPackSlab) {
          op.pair2 = variant & 2 ? 1 : 0;
          const int64_t rest = op.pair2 ? n2 * n2 : n2;
          op.i0 = n1 / 4; op.ci = n1 - n1 / 4 - (n1 > 3 ? 1 : 0);
          nx = op.ci * n1 * rest;
          int64_t e_end = op.i0 + op.ci;
          pack_rows = 0;
          for (int64_t e = op.i0; e < e_end; ++e) pack_rows += n1 - 1 - e;
          ny = pack_rows * (op.pair2 ? np2 : n2);
        }
        if (mode == SsOp::kT1T1 && !cx) continue;   // complex only
        const int npl = cx ? 2 : 1;
        std::vector<double> x(2 * nx + 1), y(2 * ny + 1);
        for (auto& v : x) v = rand() / (double)RAND_MAX - 0.5;
        for (auto& v : y) v = rand() / (double)RAND_MAX - 0.5;
        if (mode == SsOp::kMask)
          for (int64_t k = 0; k < nx; ++k) x[k] = (rand() % 3) ? 1.0 : 0.0;
        std::vector<double> xr = x, yr = y;
        auto X = [&](int pl, int64_t o) { return x[pl * nx + o]; };
        auto Y = [&](int pl, int64_t o) { return y[pl * ny + o]; };
        switch (mode) {
          case SsOp::kExpand:
            for (int64_t ii = 0; ii < ci; ++ii)
              for (int64_t jj = 0; jj < cj; ++jj)
                for (int64_t a = 0; a < n2; ++a)
                  for (int64_t b = 0; b < n2; ++b)
                    for (int pl = 0; pl < npl; ++pl) {
                      const int64_t i = i0 + ii, j = j0 + jj, o = ((ii * cj + jj) * n2 + a) * n2 + b;
                      double v = 0.0;
                      if (i != j && a != b)
                        v = op.alpha * (i < j ? 1 : -1) * (a < b ? 1 : -1) *
                            Y(pl, pidx(std::min(i, j), std::max(i, j), n1) * np2 + pidx(std::min(a, b), std::max(a, b), n2));
                      xr[pl * nx + o] = v + (beta ? X(pl, o) : 0.0);
                    }
            break;
          case SsOp::kAccum: {
            auto inI = [&](int64_t k) { return k >= i0 && k < i0 + ci; };
            auto inJ = [&](int64_t k) { return k >= j0 && k < j0 + cj; };
            auto xv = [&](int pl, int64_t i, int64_t j, int64_t a, int64_t b) {
              return X(pl, (((i - i0) * cj + (j - j0)) * n2 + a) * n2 + b);
            };
            for (int64_t k = 0; k < n1; ++k)
              for (int64_t l = k + 1; l < n1; ++l)
                for (int64_t a = 0; a < n2; ++a)
                  for (int64_t b = a + 1; b < n2; ++b)
                    for (int pl = 0; pl < npl; ++pl) {
                      double v = 0.0;
                      if (inI(k) && inJ(l)) v += xv(pl, k, l, a, b) - (anti2 ? xv(pl, k, l, b, a) : 0.0);
                      if (anti1 && inI(l) && inJ(k)) v -= xv(pl, l, k, a, b) - (anti2 ? xv(pl, l, k, b, a) : 0.0);
                      yr[pl * ny + pidx(k, l, n1) * np2 + pidx(a, b, n2)] += op.alpha * v;
                    }
            break;
          }
          case SsOp::kAccumRows:
            for (int64_t pp = 0; pp < op.ci; ++pp)
              for (int64_t a = 0; a < n2; ++a)
                for (int64_t b = a + 1; b < n2; ++b)
                  for (int pl = 0; pl < npl; ++pl)
                    yr[pl * ny + (op.i0 + pp) * np2 + pidx(a, b, n2)] +=
                        op.alpha * (X(pl, (pp * n2 + a) * n2 + b) - (anti2 ? X(pl, (pp * n2 + b) * n2 + a) : 0.0));
            break;
          case SsOp::kT1T1:
            for (int64_t i = 0; i < n1; ++i)
              for (int64_t j = i + 1; j < n1; ++j)
                for (int64_t a = 0; a < n2; ++a)
                  for (int64_t b = a + 1; b < n2; ++b) {
                    auto ur = [&](int64_t p, int64_t q) { return X(0, p * n2 + q); };
                    auto ui = [&](int64_t p, int64_t q) { return X(1, p * n2 + q); };
                    const double vr = ur(i, a) * ur(j, b) - ui(i, a) * ui(j, b) - (ur(i, b) * ur(j, a) - ui(i, b) * ui(j, a));
                    const double vi = ur(i, a) * ui(j, b) + ui(i, a) * ur(j, b) - (ur(i, b) * ui(j, a) + ui(i, b) * ur(j, a));
                    const int64_t o = pidx(i, j, n1) * np2 + pidx(a, b, n2);
                    yr[o] = op.alpha * vr + (beta ? Y(0, o) : 0.0);
                    yr[ny + o] = op.alpha * vi + (beta ? Y(1, o) : 0.0);
                  }
            break;
          case SsOp::kMask:
            for (int64_t i = 0; i < n1; ++i)
              for (int64_t j = i + 1; j < n1; ++j)
                for (int64_t a = 0; a < n2; ++a)
                  for (int64_t b = a + 1; b < n2; ++b)
                    for (int pl = 0; pl < npl; ++pl) {
                      const int64_t o = pidx(i, j, n1) * np2 + pidx(a, b, n2);
                      yr[pl * ny + o] = Y(pl, o) * x[i] * x[j] * x[n1 + a] * x[n1 + b];
                    }
            break;
          default: {   // kPackSlab
            const int64_t base = pidx(op.i0, op.i0 + 1, n1), rest = op.pair2 ? n2 * n2 : n2, nq = op.pair2 ? np2 : n2;
            for (int64_t ee = 0; ee < op.ci; ++ee)
              for (int64_t f = op.i0 + ee + 1; f < n1; ++f)
                for (int pl = 0; pl < npl; ++pl) {
                  const int64_t p = pidx(op.i0 + ee, f, n1) - base, xo = (ee * n1 + f) * rest;
                  if (op.pair2) {
                    for (int64_t a = 0; a < n2; ++a)
                      for (int64_t b = a + 1; b < n2; ++b)
                        yr[pl * ny + p * nq + pidx(a, b, n2)] = op.alpha * (X(pl, xo + a * n2 + b) - X(pl, xo + b * n2 + a));
                  } else {
                    for (int64_t c = 0; c < n2; ++c) yr[pl * ny + p * nq + c] = op.alpha * X(pl, xo + c);
                  }
                }
          }
        }
        double* dx = (double*)be->alloc(16 * nx + 16);
        double* dy = (double*)be->alloc(16 * ny + 16);
        be->h2d(dx, x.data(), 8 * x.size());
        be->h2d(dy, y.data(), 8 * y.size());
        // pair tables
        std::vector<int32_t> t(2 * np1 + 2 * np2 + 1);
        int64_t k = 0;
        for (int i = 0; i < n1; ++i) for (int j = i + 1; j < n1; ++j) { t[k] = i; t[np1 + k] = j; ++k; }
        k = 0;
        for (int a = 0; a < n2; ++a) for (int b = a + 1; b < n2; ++b) { t[2 * np1 + k] = a; t[2 * np1 + np2 + k] = b; ++k; }
        int32_t* dt = (int32_t*)be->alloc(4 * t.size());
        be->h2d(dt, t.data(), 4 * t.size());
        op.pt.oi = dt; op.pt.oj = dt + np1; op.pt.va = dt + 2 * np1; op.pt.vb = dt + 2 * np1 + np2;
        op.y_re = dy; op.y_im = cx ? dy + ny : nullptr;
        if (mode == SsOp::kT1T1) { op.u_re = dx; op.u_im = dx + nx; }
        else if (mode == SsOp::kMask) { op.m1 = dx; op.m2 = dx + n1; }
        else { op.x_re = dx; op.x_im = cx ? dx + nx : nullptr; }
        be->ss(op);
        be->sync();
        std::vector<double> xo(x.size()), yo(y.size());
        be->d2h(xo.data(), dx, 8 * x.size());
        be->d2h(yo.data(), dy, 8 * y.size());
        double e = 0.0;
        for (int64_t q = 0; q < npl * nx; ++q) e = std::fmax(e, std::fabs(xo[q] - xr[q]));
        for (int64_t q = 0; q < npl * ny; ++q) e = std::fmax(e, std::fabs(yo[q] - yr[q]));
        std::string m;
        const bool ok = e <= 1e-14 && be->ok(&m);
        ++runs;
        if (!ok) {
          ++fails;
          printf("PAIRS FAIL mode %d n1 %ld n2 %ld variant %d err %.3g %s\n", mode, (long)n1, (long)n2, variant, e,
                 m.c_str());
        }
        be->release(dx);
        be->release(dy);
        be->release(dt);
      }
  printf("pairs probe: %d runs, %d failures\n", runs, fails);
  return fails;
}

int main(int argc, char** argv) {
  std::string err;
  Backend* be = make_hip_backend(nullptr, &err);
  if (!be) { printf("no backend %s\n", err.c_str()); return 1; }
  const int f = check_permute(be) + check_pairs(be);
  return (check(be) || f) ? 2 : 0;
}
