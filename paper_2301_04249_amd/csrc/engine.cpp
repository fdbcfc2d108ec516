// Contraction planner and tensor views.
#include "engine.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace rteom {

namespace {
constexpr int64_t kComputeUnits = 256;   // MI355X
constexpr int64_t kMinSplitK = 128;      // shortest K chunk worth a work-group
constexpr int64_t kSmallK = 16;          // sums this short run on the vector units
constexpr int64_t kBatchMaxK = 1024;     // longer sums: batch a product only over nearly full tiles
constexpr int64_t kSplitMinK = 64;       // reduced precision: shortest sum whose operands are converted once
constexpr double kSplitMinMacs = 1e9;    // ... and smallest product (MACs) worth the extra pass
}  // namespace

View make_view(double* re, double* im, std::initializer_list<int64_t> dims) {
  View v;
  v.re = re;
  v.im = im;
  v.nd = static_cast<int>(dims.size());
  int d = 0;
  for (int64_t x : dims) v.dim[d++] = x;
  int64_t s = 1;
  for (int k = v.nd - 1; k >= 0; --k) {
    v.str[k] = s;
    s *= v.dim[k];
  }
  return v;
}

View reorder(const View& v, std::initializer_list<int> order) {
  View r = v;
  int d = 0;
  for (int o : order) {
    r.dim[d] = v.dim[o];
    r.str[d] = v.str[o];
    r.frac[d] = v.frac[o];
    ++d;
  }
  r.nd = d;
  return r;
}

View with_frac(View v, std::initializer_list<double> f) {
  int d = 0;
  for (double x : f) v.frac[d++] = x;
  return v;
}

View block(const View& v, std::initializer_list<int64_t> lo, std::initializer_list<int64_t> n) {
  View r = v;
  int64_t off = 0;
  int d = 0;
  auto it = n.begin();
  for (int64_t l : lo) {
    off += l * v.str[d];
    r.dim[d] = *it++;
    ++d;
  }
  r.re = v.re ? v.re + off : nullptr;
  r.im = v.im ? v.im + off : nullptr;
  return r;
}

View diagonal(const View& v, int d0, int d1) {
  View r;
  r.re = v.re;
  r.im = v.im;
  int k = 0;
  for (int d = 0; d < v.nd; ++d) {
    if (d == d1) continue;
    r.dim[k] = v.dim[d];
    r.str[k] = (d == d0) ? v.str[d0] + v.str[d1] : v.str[d];
    r.frac[k] = (d == d0) ? std::min(v.frac[d0], v.frac[d1]) : v.frac[d];
    ++k;
  }
  r.nd = k;
  return r;
}

double* Arena::take(int64_t ndoubles) {
  size_t bytes = static_cast<size_t>(ndoubles) * sizeof(double);
  bytes = (bytes + 255) & ~static_cast<size_t>(255);
  if (top_ + bytes > cap_) {
    throw Error(2, "device workspace exhausted: need " + std::to_string(top_ + bytes) +
                       " bytes, have " + std::to_string(cap_));
  }
  double* p = reinterpret_cast<double*>(base_ + top_);
  top_ += bytes;
  peak_ = std::max(peak_, top_);
  return p;
}

View Engine::temp(std::initializer_list<int64_t> dims, bool cplx) {
  int64_t n = 1;
  for (int64_t x : dims) n *= x;
  double* re = scratch->take(cplx ? 2 * n : n);
  return make_view(re, cplx ? re + n : nullptr, dims);
}

namespace {

struct Spec {
  std::string a, b, c;
};

Spec parse(const char* spec) {
  std::string s(spec);
  size_t comma = s.find(','), arrow = s.find("->");
  if (comma == std::string::npos || arrow == std::string::npos || arrow < comma)
    throw Error(1, std::string("bad contraction spec ") + spec);
  return {s.substr(0, comma), s.substr(comma + 1, arrow - comma - 1), s.substr(arrow + 2)};
}

int pos(const std::string& s, char c) {
  size_t p = s.find(c);
  return p == std::string::npos ? -1 : static_cast<int>(p);
}

// Is the index group (letters in this order) addressable with one stride in v?
bool flat(const View& v, const std::string& letters, const std::string& group, int64_t* stride) {
  int last = -1;
  int64_t s = 0;
  for (char c : group) {
    int d = pos(letters, c);
    if (v.dim[d] == 1) continue;
    if (last >= 0 && v.str[last] != v.str[d] * v.dim[d]) return false;
    last = d;
    s = v.str[d];
  }
  *stride = s;
  return true;
}

int64_t group_size(const View& v, const std::string& letters, const std::string& group) {
  int64_t n = 1;
  for (char c : group) n *= v.dim[pos(letters, c)];
  return n;
}

std::string minus(const std::string& s, char c) {
  std::string r;
  for (char x : s)
    if (x != c) r += x;
  return r;
}

}  // namespace

void Engine::add(const View& out, const View& in, double alpha_re, double alpha_im, int beta,
                 const double* const* scale_vecs) {
  if (out.nd != in.nd) throw Error(1, "add: rank mismatch");
  PermOp op;
  op.nd = out.nd;
  for (int d = 0; d < out.nd; ++d) {
    if (out.dim[d] != in.dim[d]) throw Error(1, "add: shape mismatch");
    op.dim[d] = out.dim[d];
    op.in_str[d] = in.str[d];
    op.out_str[d] = out.str[d];
    op.scale[d] = scale_vecs ? scale_vecs[d] : nullptr;
  }
  if (!out.cplx() && (in.cplx() || alpha_im != 0.0)) throw Error(1, "add: complex into real");
  op.in_re = in.re;
  op.in_im = in.im;
  op.out_re = out.re;
  op.out_im = out.im;
  op.alpha_re = alpha_re;
  op.alpha_im = alpha_im;
  op.beta = beta;
  if (!dry) {
    be->set_phase(kPhaseMove);
    be->permute(op);
    be->set_phase(phase);
  }
}

void Engine::ss(const SsOp& op) {
  if (dry) return;
  be->set_phase(kPhaseMove);
  be->ss(op);
  be->set_phase(phase);
}

void Engine::scale(const View& out, const double* const* scale_vecs) {
  add(out, out, 1.0, 0.0, 0, scale_vecs);
}

void Engine::contract(const char* spec_str, const View& A, const View& B, const View& C,
                      double alpha, int beta, ConvSlot* b_slot) {
  Spec sp = parse(spec_str);
  if ((int)sp.a.size() != A.nd || (int)sp.b.size() != B.nd || (int)sp.c.size() != C.nd)
    throw Error(1, std::string("contract: rank does not match spec ") + spec_str);
  // sizes must agree
  auto dim_of = [&](char c) -> int64_t {
    int64_t d = -1;
    int p;
    if ((p = pos(sp.a, c)) >= 0) d = A.dim[p];
    if ((p = pos(sp.b, c)) >= 0) {
      if (d >= 0 && d != B.dim[p]) throw Error(1, std::string("contract: size mismatch ") + spec_str);
      d = B.dim[p];
    }
    if ((p = pos(sp.c, c)) >= 0) {
      if (d >= 0 && d != C.dim[p]) throw Error(1, std::string("contract: size mismatch ") + spec_str);
      d = C.dim[p];
    }
    return d;
  };
  std::string Bg, Mg, Ng, Kg;
  for (char c : sp.c) {
    bool ina = pos(sp.a, c) >= 0, inb = pos(sp.b, c) >= 0;
    if (ina && inb) Bg += c;
    else if (ina) Mg += c;
    else if (inb) Ng += c;
    else throw Error(1, std::string("contract: output-only index in ") + spec_str);
  }
  for (char c : sp.a) {
    if (pos(sp.c, c) < 0) {
      if (pos(sp.b, c) < 0) throw Error(1, std::string("contract: unsummed index in ") + spec_str);
      Kg += c;
    }
  }
  for (char c : sp.b)
    if (pos(sp.c, c) < 0 && pos(sp.a, c) < 0)
      throw Error(1, std::string("contract: unsummed index in ") + spec_str);
  for (char c : sp.a + sp.b + sp.c) dim_of(c);
  const bool cplx_out = A.cplx() || B.cplx();
  if (cplx_out != C.cplx()) throw Error(1, std::string("contract: output type ") + spec_str);

  const size_t mk = scratch->mark();
  int64_t s0, s1, s2;
  // Output: direct if its batch/row/column groups are flat, possibly after
  // promoting one row or column index to a broadcast batch index.
  View Cu = C;
  std::string cl = sp.c;
  bool ctemp = false;
  bool cok = flat(C, cl, Bg, &s0) && flat(C, cl, Mg, &s1) && flat(C, cl, Ng, &s2);
  if (!cok && Bg.empty()) {
    // Fraction of the 64x64 output tiles that holds useful elements.
    auto fill = [&](const std::string& m, const std::string& n) {
      int64_t M = 1, N = 1;
      for (char c : m) M *= dim_of(c);
      for (char c : n) N *= dim_of(c);
      return static_cast<double>(M * N) / static_cast<double>(((M + 63) / 64) * 64 * ((N + 63) / 64) * 64);
    };
    for (char c : Mg + Ng) {
      std::string m2 = minus(Mg, c), n2 = minus(Ng, c), b2(1, c);
      if (flat(C, cl, b2, &s0) && flat(C, cl, m2, &s1) && flat(C, cl, n2, &s2)) {
        // promote only if the batched product fills its tiles nearly as well as
        // one product into a temporary (which costs a permute of the output); a
        // long sum makes the product compute bound, and there a batch of narrow
        // products also re-reads its operands once per batch entry, so only
        // (nearly) full tiles qualify
        int64_t K = 1;
        for (char k : Kg) K *= dim_of(k);
        const double need = K >= kBatchMaxK ? 0.95 : 0.6;
        if (fill(m2, n2) < need * fill(Mg, Ng)) continue;
        Bg = b2;
        Mg = m2;
        Ng = n2;
        cok = true;
        break;
      }
    }
  }
  if (!cok) {
    ctemp = true;
    std::string order = Bg + Mg + Ng;
    View t;
    int64_t n = 1;
    t.nd = static_cast<int>(order.size());
    for (int d = 0; d < t.nd; ++d) t.dim[d] = dim_of(order[d]);
    for (int d = t.nd - 1; d >= 0; --d) {
      t.str[d] = n;
      n *= t.dim[d];
    }
    double* p = scratch->take(cplx_out ? 2 * n : n);
    t.re = p;
    t.im = cplx_out ? p + n : nullptr;
    Cu = t;
    cl = order;
  }
  // Inputs: copy to [batch][rows][sum] / [batch][sum][cols] when not flat.
  // The product kernels address 16 rows of k and 128 rows or columns of one operand
  // through one buffer resource of at most 2 GiB: an operand whose tile would span
  // more is copied with the sum index contiguous.
  auto window_ok = [](int64_t s_mn, int64_t s_k) {
    return (127 * std::llabs(s_mn) + 15 * std::llabs(s_k) + 1) * 8 < (int64_t(1) << 31);
  };
  auto prep = [&](const View& X, const std::string& xl, const std::string& g0,
                  const std::string& g1, const std::string& g2, bool is_b, std::string* out_l) -> View {
    // batch letters missing from this operand are broadcast (stride 0)
    std::string gb;
    for (char c : g0)
      if (pos(xl, c) >= 0) gb += c;
    const std::string& gk = is_b ? g1 : g2;
    const std::string& gmn = is_b ? g2 : g1;
    int64_t t0, t1, t2;
    if (flat(X, xl, gb, &t0) && flat(X, xl, g1, &t1) && flat(X, xl, g2, &t2)) {
      int64_t sk = 0, smn = 0;
      flat(X, xl, gk, &sk);
      flat(X, xl, gmn, &smn);
      if (window_ok(smn, sk)) {
        *out_l = xl;
        return X;
      }
    }
    std::string order = gb + g1 + g2;
    if (is_b) {
      int64_t nn = 1;
      for (char c : g2) nn *= dim_of(c);
      if (!window_ok(1, nn)) order = gb + g2 + g1;   // [batch][cols][sum]
    }
    View t;
    t.nd = static_cast<int>(order.size());
    int64_t n = 1;
    for (int d = 0; d < t.nd; ++d) t.dim[d] = dim_of(order[d]);
    for (int d = t.nd - 1; d >= 0; --d) {
      t.str[d] = n;
      n *= t.dim[d];
    }
    double* p = scratch->take(X.cplx() ? 2 * n : n);
    t.re = p;
    t.im = X.cplx() ? p + n : nullptr;
    View src;
    src.re = X.re;
    src.im = X.im;
    src.nd = t.nd;
    for (int d = 0; d < t.nd; ++d) {
      int q = pos(xl, order[d]);
      src.dim[d] = X.dim[q];
      src.str[d] = X.str[q];
    }
    add(t, src, 1.0, 0.0, 0);
    *out_l = order;
    return t;
  };
  std::string al, bl;
  View Au = prep(A, sp.a, Bg, Mg, Kg, false, &al);
  View Bu = prep(B, sp.b, Bg, Kg, Ng, true, &bl);

  GemmOp op;
  op.M = 1;
  for (char c : Mg) op.M *= dim_of(c);
  op.N = 1;
  for (char c : Ng) op.N *= dim_of(c);
  op.K = 1;
  for (char c : Kg) op.K *= dim_of(c);
  op.batch = 1;
  for (char c : Bg) op.batch *= dim_of(c);
  auto strides = [&](const View& X, const std::string& xl, const std::string& g) -> int64_t {
    std::string present;
    for (char c : g)
      if (pos(xl, c) >= 0) present += c;
    int64_t s = 0;
    flat(X, xl, present, &s);
    return s;
  };
  op.a_re = Au.re;
  op.a_im = Au.im;
  op.a_sm = strides(Au, al, Mg);
  op.a_sk = strides(Au, al, Kg);
  op.a_sb = strides(Au, al, Bg);
  op.b_re = Bu.re;
  op.b_im = Bu.im;
  op.b_sk = strides(Bu, bl, Kg);
  op.b_sn = strides(Bu, bl, Ng);
  op.b_sb = strides(Bu, bl, Bg);
  op.c_re = Cu.re;
  op.c_im = Cu.im;
  op.c_sm = strides(Cu, cl, Mg);
  op.c_sn = strides(Cu, cl, Ng);
  op.c_sb = strides(Cu, cl, Bg);
  op.alpha = alpha;
  op.beta = ctemp ? 0 : beta;
  op.prec = prec;
  // Split K when that fills the device better: choose the factor whose work-group
  // count wastes the least of the last round over the compute units.
  if (op.batch == 1 && op.K > kSmallK) {
    const int64_t tiles = ((op.M + 63) / 64) * ((op.N + 63) / 64);
    double best = 0.0;
    int64_t best_s = 1;
    for (int64_t s = 1; s <= 64 && (s == 1 || op.K / s >= kMinSplitK); ++s) {
      const int64_t groups = tiles * s;
      const int64_t rounds = (groups + kComputeUnits - 1) / kComputeUnits;
      const double use = static_cast<double>(groups) / static_cast<double>(rounds * kComputeUnits);
      if (use > best + 0.05) {
        best = use;
        best_s = s;
      }
    }
    // bound the partial-sum buffer
    while (best_s > 1 && best_s * op.M * op.N * (cplx_out ? 2 : 1) * 8 > (int64_t(1) << 30)) --best_s;
    if (best_s > 1) {
      op.splitk = static_cast<int>(best_s);
      op.partial = scratch->take((cplx_out ? 2 : 1) * best_s * op.M * op.N);
    }
  }
  // Reduced precisions: large products convert their operands once (bf16 hi/lo
  // planes, or float planes) instead of in every work-group that stages them
  if (prec != 0 && op.K >= kSplitMinK && static_cast<double>(op.M) * op.N * op.K * op.batch >= kSplitMinMacs &&
      op.M >= 64 && op.N >= 64) {
    // a constant B (the caller's slot), used as it is (no copy) and alone in its batch
    // (not for fp16x3, whose planes carry per-row scales the slot does not hold)
    const bool resident = prec != 3 && b_slot && b_slot->p && op.b_im == nullptr && op.batch == 1 && Bu.re == B.re &&
                          conv_doubles(op.N, op.K) <= b_slot->doubles;
    if (resident) {
      if (b_slot->ready && (b_slot->rows != op.N || b_slot->k != op.K || b_slot->s_row != op.b_sn ||
                            b_slot->s_k != op.b_sk))
        throw Error(1, std::string("contract: converted operand layout changed in ") + spec_str);
      // the conversion is written once, outside graph capture (a discarded capture
      // would leave the slot marked but never written)
      if (!b_slot->ready && !dry && be->capturing())
        throw Error(1, std::string("contract: converted operand first used inside a graph capture in ") + spec_str);
      op.b_conv = b_slot->p;
      op.b_conv_fill = b_slot->ready ? 0 : 1;
      if (!dry) {
        b_slot->ready = true;
        b_slot->rows = op.N;
        b_slot->k = op.K;
        b_slot->s_row = op.b_sn;
        b_slot->s_k = op.b_sk;
      }
    }
    op.split = scratch->take(split_doubles(op.M, resident ? 0 : op.N, op.K, op.a_sb ? op.batch : 1,
                                           op.b_sb ? op.batch : 1, op.a_im != nullptr, op.b_im != nullptr, prec));
  } else if (prec == 3) {
    // fp16x3 is a converted-operand product only: the small ones run in float32
    op.prec = 1;   // float32
  }
  const double mult = (A.cplx() && B.cplx()) ? 4.0 : ((A.cplx() || B.cplx()) ? 2.0 : 1.0);
  const double f = 2.0 * mult * static_cast<double>(op.M) * op.N * op.K * op.batch;
  // the method's own share: every letter scaled by the smallest existing-index fraction
  // any operand gives it
  double fa = f;
  for (char c : Bg + Mg + Ng + Kg) {
    double fr = 1.0;
    int p;
    if ((p = pos(sp.a, c)) >= 0) fr = std::min(fr, A.frac[p]);
    if ((p = pos(sp.b, c)) >= 0) fr = std::min(fr, B.frac[p]);
    if ((p = pos(sp.c, c)) >= 0) fr = std::min(fr, C.frac[p]);
    fa *= fr;
  }
#ifdef RTEOM_PLAN_TRACE
  std::fprintf(stderr, "PLAN %-22s M=%lld N=%lld K=%lld batch=%lld split=%d A%s%s B%s%s ctemp=%d flops=%.3g arena=%.2fGiB\n",
               spec_str, (long long)op.M, (long long)op.N, (long long)op.K, (long long)op.batch, op.splitk,
               op.a_im ? "c" : "r", op.a_sk == 1 ? "k" : "m", op.b_im ? "c" : "r", op.b_sk == 1 ? "k" : "n",
               (int)ctemp, f, scratch->mark() / 1073741824.0);
#endif
  flops += f;
  phase_flops[phase] += f;
  alg_flops += fa;
  alg_phase_flops[phase] += fa;
  if (op.M > 0 && op.N > 0 && op.batch > 0 && !dry) {
    if (op.K == 0) {
      // empty sum: C = beta * C
      if (!op.beta) {
        View z = Cu;
        add(z, z, 0.0, 0.0, 0);
      }
    } else {
      be->gemm(op);
    }
  }
  if (ctemp) {
    View src;
    src.re = Cu.re;
    src.im = Cu.im;
    src.nd = C.nd;
    for (int d = 0; d < C.nd; ++d) {
      int q = pos(cl, sp.c[d]);
      src.dim[d] = Cu.dim[q];
      src.str[d] = Cu.str[q];
    }
    add(C, src, 1.0, 0.0, beta);
  }
  scratch->release(mk);
}

}  // namespace rteom
