// Host-side helpers shared by the C-ABI sources (api.cpp, gradient.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <functional>

#include "ovs_common.h"

namespace ovs {

// Orders the library stream after the caller's stream on entry, and the
// caller's stream after the library stream on exit.
struct StreamScope {
  ovs_lattice_s* l;
  explicit StreamScope(ovs_lattice_s* lat) : l(lat) {
    (void)hipGetLastError();  // drop a stale error left by an earlier library call (e.g. rocBLAS)
    (void)hipEventRecord(l->ev_in, l->user_stream);
    (void)hipStreamWaitEvent(l->stream, l->ev_in, 0);
  }
  ~StreamScope() {
    (void)hipEventRecord(l->ev_out, l->stream);
    (void)hipStreamWaitEvent(l->user_stream, l->ev_out, 0);
  }
};

// Bump allocator over the cached workspace (or a sizing pass with base == nullptr).
struct Arena {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

// kappa * eta^{+-}_nu (Section 1): e^{+-mu} on the time hops only.
Hop make_hop(double m_w, double mu);
// Hop coefficients and gamma5 placement of an operator.
void op_setup(const ovs_lattice_s* l, ovs_op op, Hop& h, bool& g5in, bool& g5out);
size_t elem_bytes(const ovs_lattice_s* l);
// Stencil configuration for nrhs sources (tuned, or the default).
Tuning get_tuning(const ovs_lattice_s* l, int nrhs);
// Grows the lattice's cached workspace to at least bytes.
ovs_status ensure_ws(ovs_lattice_s* l, size_t bytes);
// canonical complex128 <-> internal storage-precision fields
void pack_field(const ovs_lattice_s* l, const void* canon, void* field, int nrhs);
void unpack_field(const ovs_lattice_s* l, const void* field, void* canon, int nrhs);
// links and parameters set
bool ready(const ovs_lattice_s* l);

// roctx ranges around a call and its phases, when OVS_DEBUG_RANGES is set:
// the call's range encloses one phase range at a time.
class Ranges {
 public:
  Ranges(const ovs_lattice_s* l, const char* call);
  ~Ranges();
  void phase(const char* name);
  Ranges(const Ranges&) = delete;
  Ranges& operator=(const Ranges&) = delete;

 private:
  bool on_ = false, inner_ = false;
};

// An operator on blocks of canonical complex128 fields (device): op(in, out,
// n, warn) applies it to n fields; *warn counts fields whose application
// returned a warning.
using BlockOp = std::function<ovs_status(const void*, void*, int, int*)>;
// Options of block_krylov_eigs.  field_len: complex entries per field (0:
// 12 V, the canonical layout); largest: the nev eigenvalues of largest
// magnitude by ordinary Ritz extraction (for a shift-and-invert operator)
// instead of the smallest by harmonic extraction; start: if set, fills the
// start block (n fields) in place of the fixed splitmix vectors; progress: if
// set, called after every cycle with (restarts, largest wanted residual,
// operator applications so far); nconv: the leading wanted pairs that must
// meet tol (0: all nev; the others are returned as they stand).
struct KrylovOptions {
  long field_len = 0;
  bool largest = false;
  int nconv = 0;
  std::function<void(void*, int)> start;
  std::function<void(int, double, int)> progress;
};
// Block Arnoldi with thick restarts in Krylov-Schur form and harmonic Ritz
// extraction for the target 0 (overlap_eig.cpp): the nev eigenvalues of
// smallest magnitude (host complex128 [nev]) and, if vecs, their unit vectors
// (device [nev][field_len]); info [4] as for ovs_overlap_eigs.
ovs_status block_krylov_eigs(ovs_lattice_s* l, const BlockOp& op, int nev, int ncv, int block,
                             double tol, int max_restarts, double* lambda, void* vecs,
                             double* info, const KrylovOptions& opt = KrylovOptions());

}  // namespace ovs
