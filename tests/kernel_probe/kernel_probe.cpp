// Kernel probe (test program, GPU): the GEMM backend on every operand layout,
// complex combination, ragged size, split-K, broadcast batch and tile shape
// (forced), against host loops; tile shapes and the converted-operand paths must
// agree bitwise.  Also the permute kernels against host loops.  "bench" times the
// tile shapes on large shapes.
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
  for (int prec = 0; prec < 3; ++prec)
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
      GemmOp g; g.M=M; g.N=N; g.K=K; g.batch=B;
      g.a_sm = akc ? K : 1; g.a_sk = akc ? 1 : M; g.a_sb = bcast ? 0 : M*K;   // bcast: one A for every batch entry
      g.b_sk = bkc ? 1 : N; g.b_sn = bkc ? K : 1; g.b_sb = K*N;
      g.c_sm = N; g.c_sn = 1; g.c_sb = M*N; g.alpha = 0.75; g.beta = 1; g.prec = prec;
      double* dP = nullptr;
      if (S > 1) { dP = (double*)be->alloc(16L*S*M*N); g.splitk = S; g.partial = dP; }
      for (long b=0;b<B;++b) for (long m=0;m<M;++m) for (long n=0;n<N;++n) {
        double sr=0, si=0;
        for (long k=0;k<K;++k) {
          long ia = b*g.a_sb + m*g.a_sm + k*g.a_sk, ib = b*g.b_sb + k*g.b_sk + n*g.b_sn;
          double ar=A[ia], ai= ac? A[na+ia]:0, br=Bv[ib], bi = bc? Bv[nb+ib]:0;
          sr += ar*br - ai*bi; si += ar*bi + ai*br;
        }
        long ic = b*g.c_sb + m*g.c_sm + n*g.c_sn;
        Cref[ic] = 0.75*sr + C[ic]; Cref[nc+ic] = 0.75*si + C[nc+ic];
      }
      double *dA=(double*)be->alloc(16*na), *dB=(double*)be->alloc(16*nb), *dC=(double*)be->alloc(16*nc);
      be->h2d(dA, A.data(), 16*na); be->h2d(dB, Bv.data(), 16*nb);
      g.a_re=dA; g.a_im = ac? dA+na : nullptr; g.b_re=dB; g.b_im = bc? dB+nb : nullptr;
      g.c_re=dC; g.c_im = (ac||bc) ? dC+nc : nullptr;
      double* dS = nullptr;
      if (prec >= 1) dS = (double*)be->alloc(8 * split_doubles(M, N, K, bcast ? 1 : B, B, ac, bc, prec));
      for (int vv = -1; vv < (prec >= 1 ? 9 : 6); ++vv) {
        // prec 0: -1..5; prec 1, 2: -1..3 converted while staging, then -1..3 converted before
        const int v = (prec >= 1 && vv >= 4) ? vv - 5 : vv;
        g.split = (prec >= 1 && vv >= 4) ? dS : nullptr;
        be->force_tile(v);
        be->h2d(dC, C.data(), 16*nc);
        be->gemm(g); be->sync();
        be->d2h(Cout.data(), dC, 16*nc);
        double e=0, mx=1; long nn = (ac||bc) ? 2*nc : nc;
        for (long i=0;i<nn;++i) { e = std::fmax(e, std::fabs(Cout[i]-Cref[i])); mx = std::fmax(mx, std::fabs(Cref[i])); }
        e /= mx;
        std::string m; bool ok = be->ok(&m);
        ++runs;
        const double tol = prec == 0 ? 1e-12 : (prec == 1 ? 2e-5 : 2e-3);
        // every tile shape of one kernel family gives bitwise the same result; bf16x3
        // on converted operands runs the 32x32x16 matrix cores (another k grouping
        // than the converting 16x16x32 kernel), so it has a reference of its own
        bool same = true;
        const bool own = prec == 2 && vv >= 4;
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

// Timing of each tile shape: (M, N, K, a complex, b complex, a k-contiguous, b
// k-contiguous, largest split-K factor tried); operands hold only their real planes
// when real.
static void bench(Backend* be, int min_prec, int max_prec) {
  struct S { long M, N, K; bool ac, bc, akc, bkc; int max_split; const char* what; };
  S shapes[] = {
    {1296, 105625, 105625, true, false, true, false, 1, "alpha-beta ladder (Pef,efab->Pab)"},
    {1260, 52650, 52650, true, false, true, false, 1, "same-spin ladder in pair storage"},
    {11700, 11700, 11700, true, true, true, false, 1, "ring cc"},
    {11700, 11700, 11700, true, false, true, false, 1, "ring cr"},
    {1296, 105625, 2000, false, false, false, false, 1, "Qmj,Qbe real"},
    {1296, 11700, 105625, true, false, true, false, 1, "Z (Pef,efmb->Pmb), alpha-beta"},
    {192, 12321, 12321, true, false, true, false, 1, "formaldehyde ladder"},
  };
  for (int prec = min_prec; prec <= max_prec; ++prec)
  for (auto& s : shapes) {
    if (prec > 0 && s.max_split > 1 && s.N > 60000) continue;   // the float64 timing is the one needed
    long na = s.M * s.K, nb = s.K * s.N, nc = s.M * s.N;
    const long pa = s.ac ? 2 : 1, pb = s.bc ? 2 : 1, pc = (s.ac || s.bc) ? 2 : 1;
    double *dA = (double*)be->alloc(8 * pa * na), *dB = (double*)be->alloc(8 * pb * nb), *dC = (double*)be->alloc(8 * pc * nc);
    if (!dA || !dB || !dC) { printf("alloc failed\n"); return; }
    be->fill(dA, pa * na, 0.001); be->fill(dB, pb * nb, 0.002); be->fill(dC, pc * nc, 0.0);
    GemmOp g; g.M = s.M; g.N = s.N; g.K = s.K; g.batch = 1;
    g.a_sm = s.akc ? s.K : 1; g.a_sk = s.akc ? 1 : s.M; g.a_sb = 0;
    g.b_sk = s.bkc ? 1 : s.N; g.b_sn = s.bkc ? s.K : 1; g.b_sb = 0;
    g.c_sm = s.N; g.c_sn = 1; g.c_sb = 0; g.alpha = 1.0; g.beta = 0; g.prec = prec;
    g.a_re = dA; g.a_im = s.ac ? dA + na : nullptr; g.b_re = dB; g.b_im = s.bc ? dB + nb : nullptr;
    g.c_re = dC; g.c_im = (s.ac || s.bc) ? dC + nc : nullptr;
    const double mult = (s.ac && s.bc) ? 4.0 : ((s.ac || s.bc) ? 2.0 : 1.0);
    const double flops = 2.0 * mult * s.M * s.N * s.K;
    double* dS = nullptr;
    if (prec >= 1) { dS = (double*)be->alloc(8 * split_doubles(s.M, s.N, s.K, 1, 1, s.ac, s.bc, prec)); g.split = dS; }
    double* dP = s.max_split > 1 ? (double*)be->alloc(8 * pc * s.max_split * nc) : nullptr;
    for (int sk = 1; sk <= s.max_split; sk *= 2)
    for (int v = 0; v < (prec == 0 ? 6 : 4); ++v) {
      if (sk > 1 && v != 1 && v != 4) continue;
      g.splitk = sk;
      g.partial = sk > 1 ? dP : nullptr;
      be->force_tile(v);
      be->gemm(g); be->sync();   // warm
      auto t0 = std::chrono::steady_clock::now();
      be->gemm(g); be->sync();
      double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      printf("prec=%d tile=%d split=%d %-36s M=%ld N=%ld K=%ld  %.3f ms  %.1f TFLOP/s\n", prec, v, sk, s.what, s.M, s.N,
             s.K, sec * 1e3, flops / sec / 1e12);
      fflush(stdout);
    }
    be->force_tile(-1);
    std::string m;
    if (!be->ok(&m)) { printf("backend error %s\n", m.c_str()); return; }
    be->release(dA); be->release(dB); be->release(dC);
    if (dS) be->release(dS);
    if (dP) be->release(dP);
  }
}

// Permute check: random 4-d index orders, scales, complex/real, beta; host loops.
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

// Pair storage check: pack and unpack against host loops written from the
// definition (lexicographic pairs, sign -1 per swapped pair), every flag combination.
static int check_pairs(Backend* be) {
  int fails = 0, runs = 0;
  srand(11);
  const int64_t dims[][2] = {{1, 5}, {2, 1}, {2, 3}, {5, 17}, {7, 40}, {36, 9}};
  auto pidx = [](int64_t i, int64_t j, int64_t n) {   // position of (i < j) among the pairs of n
    int64_t p = 0;
    for (int64_t a = 0; a < i; ++a) p += n - 1 - a;
    return p + (j - i - 1);
  };
  for (auto& d : dims)
    for (int flags = 0; flags < 64; ++flags) {
      const int64_t n1 = d[0], n2 = d[1];
      const int pair2 = flags & 1, anti = (flags >> 1) & 1, mode = (flags >> 2) & 1, beta = (flags >> 3) & 1;
      const bool cx = (flags >> 4) & 1;
      const int64_t nblk = (flags >> 5) & 1 ? 2 : 1;
      const int64_t rest = pair2 ? n2 * n2 : n2, np1 = n1 * (n1 - 1) / 2, nq = pair2 ? n2 * (n2 - 1) / 2 : n2;
      const int64_t xbs = n1 * n1 * rest + 3, ybs = np1 * nq + 5;   // padded block strides
      const int64_t nx = nblk * xbs, ny = nblk * ybs;
      std::vector<double> x(2 * nx), y(2 * ny), xr, yr;
      for (auto& v : x) v = rand() / (double)RAND_MAX - 0.5;
      for (auto& v : y) v = rand() / (double)RAND_MAX - 0.5;
      xr = x;
      yr = y;
      const double alpha = 0.625;
      for (int64_t b = 0; b < nblk; ++b)
        for (int64_t i = 0; i < n1; ++i)
          for (int64_t j = 0; j < n1; ++j)
            for (int64_t c = 0; c < rest; ++c) {
              const int64_t a2 = pair2 ? c / n2 : 0, b2 = pair2 ? c % n2 : c;
              const int64_t xo = b * xbs + (i * n1 + j) * rest + c;
              for (int pl = 0; pl < (cx ? 2 : 1); ++pl) {
                if (mode == 0) {
                  if (i >= j || (pair2 && a2 >= b2)) continue;
                  const int64_t yo = b * ybs + pidx(i, j, n1) * nq + (pair2 ? pidx(a2, b2, n2) : b2);
                  const int64_t xs = b * xbs + (j * n1 + i) * rest + c;
                  yr[pl * ny + yo] = alpha * (x[pl * nx + xo] - (anti ? x[pl * nx + xs] : 0.0));
                } else {
                  double v = beta ? x[pl * nx + xo] : 0.0;
                  if (i != j && !(pair2 && a2 == b2)) {
                    const int64_t q = pair2 ? pidx(std::min(a2, b2), std::max(a2, b2), n2) : b2;
                    const double sg = (i < j ? 1.0 : -1.0) * (pair2 && b2 < a2 ? -1.0 : 1.0);
                    v += alpha * sg * y[pl * ny + b * ybs + pidx(std::min(i, j), std::max(i, j), n1) * nq + q];
                  }
                  xr[pl * nx + xo] = v;
                }
              }
            }
      double* dx = (double*)be->alloc(16 * nx + 8);
      double* dy = (double*)be->alloc(16 * ny + 8);
      be->h2d(dx, x.data(), 16 * nx);
      be->h2d(dy, y.data(), 16 * ny);
      PairOp op;
      op.n1 = n1; op.n2 = n2; op.nblk = nblk; op.pair2 = pair2; op.anti = anti; op.mode = mode; op.beta = beta;
      op.alpha = alpha;
      op.x_re = dx; op.x_im = cx ? dx + nx : nullptr; op.x_bs = xbs;
      op.y_re = dy; op.y_im = cx ? dy + ny : nullptr; op.y_bs = ybs;
      be->pairs(op);
      be->sync();
      std::vector<double> xo(2 * nx), yo(2 * ny);
      be->d2h(xo.data(), dx, 16 * nx);
      be->d2h(yo.data(), dy, 16 * ny);
      double e = 0.0;
      for (int64_t k = 0; k < 2 * nx; ++k) e = std::fmax(e, std::fabs(xo[k] - xr[k]));
      for (int64_t k = 0; k < 2 * ny; ++k) e = std::fmax(e, std::fabs(yo[k] - yr[k]));
      std::string m;
      const bool ok = e <= 1e-15 && be->ok(&m);
      ++runs;
      if (!ok) {
        ++fails;
        printf("PAIRS FAIL n1 %ld n2 %ld flags %d err %.3g %s\n", (long)n1, (long)n2, flags, e, m.c_str());
      }
      be->release(dx);
      be->release(dy);
    }
  printf("pairs probe: %d runs, %d failures\n", runs, fails);
  return fails;
}

int main(int argc, char** argv) {
  std::string err;
  Backend* be = make_hip_backend(nullptr, &err);
  if (!be) { printf("no backend %s\n", err.c_str()); return 1; }
  if (argc > 1 && std::string(argv[1]) == "bench") {   // bench [lowest precision [highest precision]]
    const int lo = argc > 2 ? atoi(argv[2]) : 0;
    bench(be, lo, argc > 3 ? atoi(argv[3]) : (argc > 2 ? lo : 2));
    return 0;
  }
  const int f = check_permute(be) + check_pairs(be);
  return (check(be) || f) ? 2 : 0;
}
