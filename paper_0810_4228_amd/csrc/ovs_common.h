// Internal declarations shared by the ovsign HIP sources.
//
// Device layouts (private to the library):
//   field  : [nrhs][6][Vs][2] complex: component c = 3*spin + colour of site s
//            at ((c/2)*Vs + s)*2 + c%2 (fidx), so the two components of a pair
//            are adjacent and one 16-byte load brings both in FP32.  Complex is
//            double2 (OVS_F64) or float2 (OVS_F32_STORE).  Vs = V rounded up to
//            a wave plus one wave, so pair planes are not a power of two apart
//            (L2 set aliasing); pad entries s >= V are kept zero.
//   links  : [4][5][Vs][2] complex: entry e = 3*a + b of U_{x,nu} at
//            ((nu*5 + e/2)*Vs + s)*2 + e%2 (lidx); the second slot of pair 4
//            is zero.  The boundary sign of the link leaving the last slice in
//            direction nu is folded in.
//   FP64 work fields (deflation, results): the field layout in double2
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/ovsign.h"

namespace ovs {

constexpr int kWG = 256;          // workgroup size of the streaming kernels
constexpr int kLinkSlots = 10;    // complex slots per site and direction (9 entries + 1 pad)

// Offset of component c of site s in one source field (complex elements).
__host__ __device__ inline long fidx(int c, long s, long Vs) {
  return ((long)(c >> 1) * Vs + s) * 2 + (c & 1);
}
// Offset of entry e of U_nu at site s in the packed links (complex elements).
__host__ __device__ inline long lidx(int nu, int e, long s, long Vs) {
  return ((long)(nu * 5 + (e >> 1)) * Vs + s) * 2 + (e & 1);
}
constexpr int kMaxNrhs = 4096;
constexpr int kMaxDefl = 1024;

struct Geometry {
  int lx, ly, lz, lt;
  int V;
  int Vs;   // padded stride of one component plane (V rounded up, plus one wave)
};

// Hop coefficients kappa*eta_nu^{+-} for one operator application.
struct Hop {
  float f32_fwd[4], f32_bwd[4];
  double fwd[4], bwd[4];
};

struct Tuning {
  int rhs_block = 1;     // sources per thread in the stencil
  int wg = 256;          // stencil workgroup size
  int lds_kb = 0;        // dynamic LDS per workgroup (KiB): caps workgroups per CU
  int order = 0;         // 0: source blocks of a tile adjacent, 1: source block slowest
  int g = 1;             // lanes sharing one site (each lane one source); 1 = source blocking
  int nt = 0;            // streaming (non-temporal) stores of the output
  int stage = 0;         // 1: the tile's input spinors staged in LDS (g = 1 only)
  bool tuned = false;
};

// Per-source Krylov coefficients, device resident.  Index i is 0-based
// (entry i describes Lanczos vector i+1 of the paper's numbering).
struct CoefArrays {
  double2* alpha;   // [nrhs][kmax]
  double* beta;     // [nrhs][kmax]
  double2* gamma;   // [nrhs][kmax]
  double* sv;       // [nrhs][kmax+1] scale of stored v (v_i = sv_i * V~_i)
  double2* sw;      // [nrhs][kmax+1] scale of stored w (w_i = sw_i * W~_i)
  double* tnorm2;   // [nrhs][kmax]  |A v_i|^2
  int* kstop;       // [nrhs] number of valid alpha (kmax if no breakdown)
  int* status;      // [nrhs] 0 ok, 1 lucky, 2 serious
  int kmax;
  double* dnorm = nullptr;  // [nrhs][kmax] |delta_i| / (|v~| |w~|) of each beta step, or null
  int inject_plus1 = 0;     // > 0: the beta step of iteration inject_plus1 - 1 takes delta
                            // as zero (a serious breakdown forced from the host, for tests)
};

}  // namespace ovs

struct ovs_lattice_s {
  ovs::Geometry g;
  int bc[4];
  ovs_precision prec;
  hipStream_t user_stream;      // caller's stream (may be the NULL stream)
  hipStream_t stream;           // library stream (non-blocking, default priority)
  hipEvent_t ev_in, ev_out;     // ordering with the caller's stream
  int device;
  double m_w = -1.5, mu = 0.0;
  bool params_set = false;
  bool links_set = false;
  void* links = nullptr;        // packed links, storage precision
  void* links64 = nullptr;      // FP64 copy for the eigensolver (FP32 lattices only)
  // tuned stencil configuration per nrhs
  std::vector<std::pair<int, ovs::Tuning>> tuning;
  // tuned dual-stencil configuration per nrhs (wg unused: always 256)
  std::vector<std::pair<int, ovs::Tuning>> dual_tuning;
  int lds_max_kb = 64;          // largest dynamic LDS request the device accepts
  // OVS_DEBUG_* flags and the iteration whose delta is forced to zero (-1: none)
  int debug_flags = 0;
  int debug_breakdown_at = -1;
  // cached workspace for sign_apply and apply
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // cached one-pass Lanczos basis (grown as a solve needs it)
  void* bbuf = nullptr;
  size_t bbuf_bytes = 0;
  // results of the last sign_apply (host copies) for diagnostics
  std::vector<double> last_alpha, last_beta, last_gamma, last_x;
  int last_nrhs = 0, last_kmax = 0;
  // FP64 handle for sources whose tolerance is below the FP32 storage floor
  // (FP32 lattices only): shares links64, the stream and the parameters.
  ovs_lattice_s* shadow64 = nullptr;
  ovs_lattice_s* parent = nullptr;   // set on a shadow: the handle it serves
  void* split_buf = nullptr;         // gathered sources / results of the split
  size_t split_bytes = 0;
  // second handle (own stream) for the concurrent half of large batches
  ovs_lattice_s* worker = nullptr;
  // recorded on this handle's stream before the worker half starts: the
  // worker's stream waits on it, so work already enqueued here (e.g. a gather
  // of the sources into split_buf) is complete before the worker reads it
  hipEvent_t ev_fork = nullptr;
};

struct ovs_field_s {
  ovs_lattice_s* lat;
  int nrhs;
  void* data;   // [nrhs][12][V] storage-precision complex
};

struct ovs_deflation_s {
  ovs_lattice_s* lat;
  int m;
  std::vector<double> lambda;   // host complex [m]
  double2* R;                    // device [m][12][Vs]
  double2* L;                    // device [m][12][Vs]
  double* sgn;                   // device [m] sgn(Re lambda)
  double info[3] = {0, 0, 0};    // computed: max residual, max |L^dag R - I|, restarts
};

// ---- launchers implemented in stencil.hip --------------------------------
namespace ovs {

// canonical complex128 [nrhs][V][12]  <->  internal [nrhs][12][V]
void launch_pack_f64(const double2* canon, double2* field, int nrhs, const Geometry& g, hipStream_t s);
void launch_pack_f32(const double2* canon, float2* field, int nrhs, const Geometry& g, hipStream_t s);
void launch_unpack_f64(const double2* field, double2* canon, int nrhs, const Geometry& g, hipStream_t s);
void launch_unpack_f32(const float2* field, double2* canon, int nrhs, const Geometry& g, hipStream_t s);
// zero the pad entries [V, Vs) of nplanes component planes
void launch_zero_pad(void* base, bool f32, long nplanes, const Geometry& g, hipStream_t s);
void launch_pack_links(const double2* canon, void* links, bool f32, const Geometry& g,
                       const int bc[4], hipStream_t s);

// out = op in on fields of nrhs sources; g5in/g5out select gamma5 factors.
hipError_t launch_wilson(bool f32, const void* links, const void* in, void* out, int nrhs,
                         const Geometry& g, const Hop& hop, bool g5in, bool g5out,
                         const Tuning& tn, hipStream_t s);
// Lets kernels request dynamic LDS above the default per-workgroup limit.
void set_lds_limit(int kb);

// Dual stencil of the two-sided Lanczos step: for iteration i = *it,
//   T = A V~_i, S = A^dagger W~_i (A = gamma5 Dw(mu)), plus per-workgroup
//   partials of W~_i^dagger T (complex) and |T|^2 per source slot.
// V~_i = basis[ring ? i%3 : i], W~_i = wbuf[i%3]; each holds nrhs_slots
// fields; only the slots listed in rhs_map[0..*n_active) are processed.
struct DualArgs {
  const void* links;
  const void* basis;
  const void* wbuf;
  long basis_stride;   // elements between consecutive basis (or wbuf) entries
  bool ring;
  const int* it;
  void* out_t;
  void* out_s;
  double* partials;    // [slot][dual_num_wg][3]
  const int* rhs_map;
  const int* n_active;
  int nrhs_slots;
  int lds_kb;          // occupancy cap, as in Tuning
  int order;
  int nt;              // streaming stores of T and S
  int pair = 0;        // 1: lane pairs split the two operators (k_dual_pair);
                       // 2: the same with the tile's spinors staged in LDS;
                       // 3: one operator per workgroup (k_dual_op); 4: the
                       // same with the tile's spinors staged in LDS; 5: one
                       // operator and source per workgroup marching along t
                       // (k_dual_march; order 0 or 1)
  int tile = 256;      // sites per tile of k_dual (pair 0): 256, or 64 for small
                       // lattices (more workgroups); the other variants need 256;
                       // partials are [slot][ceil(V / tile)][3]
};
hipError_t launch_dual(bool f32, const DualArgs& a, const Geometry& g, const Hop& hA,
                       const Hop& hAd, int rhs_block, hipStream_t s);
int dual_num_wg(const Geometry& g);

// Persistent two-sided Lanczos: nit full iterations (dual stencil of the
// operator-per-workgroup form, alpha, update, beta with probe gather) in one
// cooperative launch; *it advances by nit.
struct PersistArgs {
  const void* links;
  void* basis;
  void* wbuf;
  long basis_stride;
  bool ring;
  int* it;
  void* T;
  void* S;
  double* part1;       // dual partials [slot][dual_num_wg][3]
  double* part2;       // update partials [slot][update_nwg][4]
  const int* rhs_map;
  const int* n_active;
  int nslots;
  int rhs_block;       // sources per thread of the dual stencil (1, 2; FP64: 1)
  bool stage;          // tile staged in LDS
  int order;
  int nt_dual;         // streaming stores of T and S
  int nt_update;       // streaming stores of the new vectors
  CoefArrays co;
  const int* idx;      // probe positions (probes != nullptr)
  int P;
  double2* probes;
  int nit;
  unsigned* bar;       // kPersistBarWords barrier words, zero before the first launch
};
constexpr int kPersistBarWords = 352;
constexpr int kPersistBarErr = 320;  // nonzero: a barrier wait ran out of polls
hipError_t launch_persistent(bool f32, const PersistArgs& a, const Geometry& g, const Hop& hA,
                             const Hop& hAd, hipStream_t s);

}  // namespace ovs

// ---- error helpers --------------------------------------------------------
namespace ovs {
// Records the failing runtime call for ovs_last_error (per host thread).
void record_error(const char* what, int line, hipError_t e);
}
#define OVS_HIP(call)                                           \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) {                                     \
      ovs::record_error(#call, __LINE__, e_);                   \
      return OVS_ERR_HIP;                                       \
    }                                                           \
  } while (0)
