// Tensor views, device arena and the contraction planner of the RT-EOM-CCSD engine.
#pragma once

#include <cstdint>
#include <initializer_list>
#include <stdexcept>
#include <string>
#include <vector>

#include "backend.h"

namespace rteom {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// A strided view of a real or planar-complex tensor in device memory.  frac[d] is the
// fraction of dimension d's indices that exist in the method (the extended orbital space
// pads each spin's occupied and virtual range to a common size); the flop count of the
// method's own work scales each summed, row or column index by it.
struct View {
  double* re = nullptr;
  double* im = nullptr;
  int nd = 0;
  int64_t dim[kMaxDims] = {0};
  int64_t str[kMaxDims] = {0};
  double frac[kMaxDims] = {1, 1, 1, 1, 1, 1};
  bool cplx() const { return im != nullptr; }
  int64_t numel() const {
    int64_t n = 1;
    for (int d = 0; d < nd; ++d) n *= dim[d];
    return n;
  }
};

// Contiguous row-major view.
View make_view(double* re, double* im, std::initializer_list<int64_t> dims);
// Reorder the dimensions of a view: result dim d is v's dim order[d].
View reorder(const View& v, std::initializer_list<int> order);
// Sub-block: dimension d restricted to [lo[d], lo[d] + n[d]).
View block(const View& v, std::initializer_list<int64_t> lo, std::initializer_list<int64_t> n);
// Diagonal of dimensions d0 and d1 (merged into d0, d1 removed).
View diagonal(const View& v, int d0, int d1);
// The same view with existing-index fractions set per dimension.
View with_frac(View v, std::initializer_list<double> f);

// Bump allocator over one device buffer; temporaries are released in LIFO order.
// All device work is ordered on one stream, so memory released after an
// operation has been enqueued may be reused by the next operation.
class Arena {
 public:
  void init(char* base, size_t bytes) { base_ = base; cap_ = bytes; top_ = 0; peak_ = 0; }
  double* take(int64_t ndoubles);
  size_t mark() const { return top_; }
  void release(size_t m) { top_ = m; }
  size_t peak() const { return peak_; }
  size_t capacity() const { return cap_; }
  void set_counting(bool c) { counting_ = c; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, top_ = 0, peak_ = 0;
  bool counting_ = false;
};

// Resident converted copy of a constant real B operand (reduced precisions): the
// first product that uses it converts B into it, later products with the same B
// layout read it as it is.
struct ConvSlot {
  double* p = nullptr;
  int64_t doubles = 0;
  bool ready = false;
  int64_t rows = 0, k = 0, s_row = 0, s_k = 0;   // layout it holds once ready
};

class Engine {
 public:
  Backend* be = nullptr;
  Arena* scratch = nullptr;
  int prec = 0;
  double flops = 0.0;       // accumulated GEMM flops (real-flop convention), as executed
  double phase_flops[kNumPhases] = {0};
  double alg_flops = 0.0;   // the same over existing spin-orbitals only (no padding)
  double alg_phase_flops[kNumPhases] = {0};
  int phase = kPhaseGemm;
  void set_phase(int ph) {
    phase = ph;
    if (!dry && be) be->set_phase(ph);
  }
  bool dry = false;          // plan only (workspace query): count scratch, issue nothing

  // C[spec_c] = alpha * sum A[spec_a] B[spec_b] + beta * C
  // spec: "ijef,efab->ijab".  Letters shared by A, B and C are batch indices,
  // A&C: rows, B&C: columns, A&B: summed.  Operands whose index groups cannot be
  // flattened to single strides are copied to a temporary first.
  void contract(const char* spec, const View& A, const View& B, const View& C, double alpha,
                int beta, ConvSlot* b_slot = nullptr);
  // out = alpha * in + beta * out (same shape), optional per-dimension scale vectors
  void add(const View& out, const View& in, double alpha_re, double alpha_im, int beta,
           const double* const* scale = nullptr);
  // same-spin pair storage operations (SsOp)
  void ss(const SsOp& op);
  // out *= prod_d scale_d (in place)
  void scale(const View& out, const double* const* scale);
  View temp(std::initializer_list<int64_t> dims, bool cplx);
};

}  // namespace rteom
