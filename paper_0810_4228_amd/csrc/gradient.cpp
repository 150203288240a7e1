// ovs_sign_apply_vjp: the gradient of L = sum_r Re <chi_r, y_r> with
// y_r = |b_r| V_k sgn(G_k) e_1 (two-sided Lanczos of Section 4 at fixed k)
// with respect to the sources b, the chemical potential mu and the links U;
// with m LR-deflation eigentriples (Section 3) y_r = R S L^dagger b_r +
// |b_R| V_k sgn(G_k) e_1 from the starts b_R = (1 - R L^dagger) b_r,
// b_L = (1 - L R^dagger) b_r.
//
// Deflated gradient.  With A = sum_k lambda_k r_k l_k^dagger, c = L^dagger b,
// s_j = sgn Re lambda_j and g_j(z) = (sgn z - s_j) / (z - lambda_j) (zero
// where sgn z = s_j), the Daleckii-Krein form of d sgn(A) splits
// dL = Re chi^dagger d sgn(A) b into
//   (i)   the complement block, the Krylov derivative of the deflated run
//         with the operator taken as Q A Q (Q = 1 - R L^dagger): the forces
//         Re <tbar, dA v> and Re <sbar, dA^dagger w> of the sweep act through
//         Q^dagger tbar and Q sbar;
//   (ii)  sum_j Re <(r_j^dagger chi) l_j, dA g_j(A) b_R>, with g_j(A) b_R =
//         |b_R| V_k g_j(G_k) e_1 = |b_R| V_k (G_k - lambda_j)^{-1} (x - s_j e_1)
//         taken from the same basis, so that it joins the force of step i as
//         the extra vector sum_j conj(|b_R| z_ji) (r_j^dagger chi) l_j;
//   (iii) sum_j Re <conj(c_j) q_j, dA r_j>, q_j = g_j(A)^dagger chi: the
//         deflated part sum_{k != j} l_k (s_k - s_j) / (conj lambda_k -
//         conj lambda_j) (r_k^dagger chi) in closed form, the complement part
//         by a second two-sided Lanczos run on A^dagger from Q^dagger chi (left
//         start Q chi) as |.| V' (G' - conj lambda_j)^{-1} (sgn(G') e_1 - s_j e_1).
// The eigentriples are those of A at the current (mu, U); the sources enter
// through grad_b = Q^dagger bbar_R + Q bbar_L + L S R^dagger chi.
//
// Forward: the recurrences (4.1)-(4.4) in FP64.  By default only checkpoints
// are kept: the pairs (v_{jc-1}, v_{jc}), (w_{jc-1}, w_{jc}) every c = ceil(sqrt k)
// steps; the reverse sweep replays each segment forward from its checkpoint
// with the stored coefficients (the same kernels and coefficient arithmetic as
// the forward pass, so the replayed vectors are bitwise those of the forward)
// and then walks it backwards.  Memory: about 4k/c + 2c + 18 fields per
// source instead of 2k + 18; cost: one more forward pass.  With
// OVS_VJP_STORE_BASIS both bases are kept instead.
// Inner sign: sgn(G_k) e_1 and its vector-Jacobian product from the same
// tau = e^u trapezoid rule, step h halved until two levels agree.  Reverse
// sweep: per iteration linear-combination passes with fused dots, two scalar
// steps, the stencil adjoints A^dagger tbar and A sbar, and the link-force
// accumulation (grad.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

#include "ovs_common.h"
#include "ovs_grad.h"
#include "ovs_host.h"
#include "ovs_krylov.h"

using namespace ovs;

namespace {

constexpr double kVjpULo = -40.0, kVjpUHi = 45.0;  // u range of the tau = e^u rule
constexpr double kVjpHStart = 0.25, kVjpHMin = 1.0 / 32.0;
constexpr double kVjpAccept = 1e-10;  // relative change between two step levels

void vjp_range(double h, int& n0, int& nnode) {
  n0 = (int)std::floor(kVjpULo / h);
  nnode = (int)std::ceil(kVjpUHi / h) - n0 + 1;
}

double max_rel_change(const std::vector<double2>& a, const std::vector<double2>& b) {
  double num = 0.0, den = 0.0;
  for (size_t i = 0; i < a.size(); ++i) {
    num = std::max(num, std::hypot(a[i].x - b[i].x, a[i].y - b[i].y));
    den = std::max(den, std::hypot(a[i].x, a[i].y));
  }
  return den > 0.0 ? num / den : num;
}

using cd = std::complex<double>;

// z = (T - shift)^{-1} rhs for the tridiagonal T (diagonal d, T(i+1,i) = lo_i,
// T(i,i+1) = up_i), Gaussian elimination with partial pivoting; false if a
// pivot vanishes.
bool tri_solve(int n, const cd* d, const cd* lo, const cd* up, cd shift, std::vector<cd>& z) {
  std::vector<cd> D(n), DU(std::max(n - 1, 1)), DL(std::max(n - 1, 1)), DU2(std::max(n - 1, 1), 0.0);
  for (int i = 0; i < n; ++i) D[i] = d[i] - shift;
  for (int i = 0; i + 1 < n; ++i) {
    DU[i] = up[i];
    DL[i] = lo[i];
  }
  for (int i = 0; i + 1 < n; ++i) {
    if (std::abs(D[i]) >= std::abs(DL[i])) {
      if (D[i] == 0.0) return false;
      const cd f = DL[i] / D[i];
      D[i + 1] -= f * DU[i];
      z[i + 1] -= f * z[i];
    } else {  // rows i and i + 1 interchanged
      const cd f = D[i] / DL[i];
      D[i] = DL[i];
      const cd t = D[i + 1];
      D[i + 1] = DU[i] - f * t;
      if (i + 2 < n) {
        DU2[i] = DU[i + 1];
        DU[i + 1] = -f * DU[i + 1];
      }
      DU[i] = t;
      std::swap(z[i], z[i + 1]);
      z[i + 1] -= f * z[i];
    }
  }
  if (D[n - 1] == 0.0) return false;
  z[n - 1] /= D[n - 1];
  if (n > 1) z[n - 2] = (z[n - 2] - DU[n - 2] * z[n - 1]) / D[n - 2];
  for (int i = n - 3; i >= 0; --i) z[i] = (z[i] - DU[i] * z[i + 1] - DU2[i] * z[i + 2]) / D[i];
  return true;
}

}  // namespace

// The vjp proper; with ws_query != NULL only the workspace it needs is
// computed (the other pointers are not used).
static ovs_status vjp_impl(ovs_lattice l, ovs_deflation defl, int32_t n_defl, const void* b,
                           const void* chi, int32_t nrhs, int32_t k, int32_t flags, void* y,
                           void* grad_b, double* grad_mu, void* grad_U, double* quad_err,
                           void* user_ws, size_t user_ws_bytes, size_t* ws_query) {
  if (!l || (!ws_query && (!b || !chi || !grad_b || !grad_mu || !grad_U))) return OVS_ERR_ARG;
  if (nrhs < 1 || nrhs > kMaxNrhs || k < 1 || k > 65535) return OVS_ERR_ARG;
  if (n_defl < 0 || (n_defl > 0 && (!defl || defl->lat != l || n_defl > defl->m)))
    return OVS_ERR_ARG;
  const int md = n_defl;  // deflated eigentriples (0: none)
  if (flags & ~OVS_VJP_STORE_BASIS) return OVS_ERR_ARG;
  if (l->prec != OVS_F64 || l->parent) return OVS_ERR_ARG;
  if (!ws_query && !ready(l)) return OVS_ERR_STATE;
  const bool store = (flags & OVS_VJP_STORE_BASIS) != 0;
  const Geometry& g = l->g;
  const long F = 12L * g.Vs;        // elements of one source field
  const long NF = (long)nrhs * F;   // elements of one batch of fields
  const int nch = lin_nchunk(F);
  const int cseg = store ? k : std::max(1, (int)std::ceil(std::sqrt((double)k)));
  const int nseg = (k + cseg - 1) / cseg;
  int n0max, nnmax;
  vjp_range(kVjpHMin, n0max, nnmax);
  constexpr int kFields = 18;

  // ---- workspace ----
  struct Ptrs {
    double2 *V, *W, *ckV, *ckW, *fld[kFields], *Fg;
    double *parts, *fparts, *gmu;
    void* vjp;
    IsignVjpOut vo[2];
    // deflation: projected sources and chi, projected forces, the second run
    // on A^dagger (full basis V2, ring W2), its coefficients
    double2 *BR, *BL, *YEX, *CHIL, *CHIR, *YCHI, *TBp, *WTBp, *V2, *W2, *QJ;
    double *CDb, *CDchi, *CDt, *dpart;
    double2 *kappa, *coefQ, *coefL;
    int* kused;
    // paired stencil (T = A x, S = A^dagger y in one launch): iteration 0,
    // active count, identity source map; per-tile partials (not used)
    int* dints;
    double* dpart2;
    // the projected tbar_i and sbar_i of the steps of one force group
    double2 *GT, *GS;
  } P_{};
  GradScalars S{}, S2{};
  // tile of the paired stencil: 64 sites on small lattices, where 256-site
  // tiles would leave most CUs idle
  const int dual_tile = (g.V / 256 < 128) ? 64 : 256;
  // force groups: the link force of cg consecutive reverse steps is summed in
  // one pass (steps i with i / cg equal; the recomputation segments, in both
  // modes, so the sums are the same)
  const int cg = std::max(1, (int)std::ceil(std::sqrt((double)k)));
  auto carve_scalars = [&](Arena& a, GradScalars& Sx) {
    const size_t nk = (size_t)nrhs * k;
    Sx.alpha = a.take<double2>(nk);
    Sx.beta = a.take<double>(nk);
    Sx.gamma = a.take<double2>(nk);
    Sx.tnorm2 = a.take<double>(nk);
    Sx.x = a.take<double2>(nk);
    Sx.xbar = a.take<double2>(nk);
    Sx.abar = a.take<double2>(nk);
    Sx.bbar = a.take<double>(nk);
    Sx.gbar = a.take<double2>(nk);
    Sx.nb = a.take<double>(nrhs);
    Sx.sigma = a.take<double2>(nrhs);
    Sx.status = a.take<int>(nrhs);
    Sx.coef = a.take<double2>((size_t)kCoefTables * kLinTerms * nrhs);
    Sx.kmax = k;
    Sx.nrhs = nrhs;
  };
  auto carve = [&](Arena& a) {
    if (store) {
      P_.V = a.take<double2>((size_t)k * NF);
      P_.W = a.take<double2>((size_t)k * NF);
    } else {
      P_.V = a.take<double2>((size_t)(cseg + 2) * NF);   // segment buffer (forward ring)
      P_.W = a.take<double2>((size_t)(cseg + 2) * NF);
      P_.ckV = a.take<double2>((size_t)2 * nseg * NF);
      P_.ckW = a.take<double2>((size_t)2 * nseg * NF);
    }
    for (int j = 0; j < kFields; ++j) P_.fld[j] = a.take<double2>(NF);
    P_.Fg = a.take<double2>(5L * 9 * g.Vs);
    carve_scalars(a, S);
    P_.parts = a.take<double>((size_t)4 * nrhs * nch * 2 * kLinDots);
    P_.fparts = a.take<double>((size_t)(g.V + kWG - 1) / kWG + 1);
    P_.gmu = a.take<double>(1);
    P_.GT = a.take<double2>((size_t)cg * NF);
    P_.GS = a.take<double2>((size_t)cg * NF);
    P_.dints = a.take<int>(2 + (size_t)nrhs);
    P_.dpart2 = a.take<double>((size_t)nrhs * ((g.V + dual_tile - 1) / dual_tile) * 3);
    P_.vjp = a.take<char>(isign_vjp_scratch_bytes(k, nnmax));
    for (int lv = 0; lv < 2; ++lv) {
      P_.vo[lv].x = a.take<double2>(k);
      P_.vo[lv].gd = a.take<double2>(k);
      P_.vo[lv].gsub_re = a.take<double>(k);
      P_.vo[lv].gsup = a.take<double2>(k);
    }
    if (md > 0) {
      for (double2** f : {&P_.BR, &P_.BL, &P_.YEX, &P_.CHIL, &P_.CHIR, &P_.YCHI, &P_.TBp, &P_.WTBp})
        *f = a.take<double2>(NF);
      P_.V2 = a.take<double2>((size_t)k * NF);
      P_.W2 = a.take<double2>((size_t)3 * NF);
      P_.QJ = a.take<double2>(F);
      carve_scalars(a, S2);
      for (double** c : {&P_.CDb, &P_.CDchi, &P_.CDt})
        *c = a.take<double>((size_t)md * nrhs * 4);
      P_.dpart = a.take<double>((size_t)md * nrhs * defl_nchunk(F) * 4);
      P_.kappa = a.take<double2>((size_t)k * nrhs * md);
      P_.coefQ = a.take<double2>((size_t)md * k * nrhs);
      P_.coefL = a.take<double2>((size_t)md * md);
      P_.kused = a.take<int>(2);
    }
  };
  Arena sizing{nullptr};
  carve(sizing);
  if (ws_query) {
    *ws_query = sizing.off + 512;
    return OVS_OK;
  }
  char* ws_base;
  if (user_ws) {
    if (user_ws_bytes < sizing.off + 512) return OVS_ERR_ARG;
    ws_base = (char*)(((uintptr_t)user_ws + 255) & ~uintptr_t(255));
  } else {
    ovs_status st0 = ensure_ws(l, sizing.off + 256);
    if (st0 != OVS_OK) return st0;
    ws_base = (char*)l->ws;
  }
  ovs_status st = OVS_OK;
  StreamScope scope(l);
  Ranges rg(l, "ovs_sign_apply_vjp");
  rg.phase("forward");
  Arena arena{ws_base};
  carve(arena);
  double2** fld = P_.fld;
  double2 *B = fld[0], *CHI = fld[1], *T = fld[2], *Sv = fld[3];
  double2* VB[2] = {fld[4], fld[5]};
  double2* WB[2] = {fld[6], fld[7]};
  double2* VTB[2] = {fld[8], fld[9]};
  double2* WTB[2] = {fld[10], fld[11]};
  double2 *TB = fld[12], *T1 = fld[13], *T2 = fld[14], *GB = fld[15], *TL = fld[16],
          *YA = fld[17];
  double* P[4];
  for (int j = 0; j < 4; ++j) P[j] = P_.parts + (size_t)j * nrhs * nch * 2 * kLinDots;

  // every field starts at zero (pads stay zero: the stencil writes sites < V only)
  OVS_HIP(hipMemsetAsync(P_.V, 0, (size_t)((char*)(fld[kFields - 1] + NF) - (char*)P_.V),
                         l->stream));
  if (md > 0) {
    for (double2* f : {P_.BR, P_.BL, P_.YEX, P_.CHIL, P_.CHIR, P_.YCHI, P_.TBp, P_.WTBp})
      OVS_HIP(hipMemsetAsync(f, 0, sizeof(double2) * NF, l->stream));
    OVS_HIP(hipMemsetAsync(P_.V2, 0, sizeof(double2) * (size_t)k * NF, l->stream));
    OVS_HIP(hipMemsetAsync(P_.W2, 0, sizeof(double2) * 3 * NF, l->stream));
    OVS_HIP(hipMemsetAsync(P_.QJ, 0, sizeof(double2) * F, l->stream));
    OVS_HIP(hipMemsetAsync(S2.xbar, 0, sizeof(double2) * (size_t)nrhs * k, l->stream));
  }
  OVS_HIP(hipMemsetAsync(P_.Fg, 0, sizeof(double2) * 5 * 9 * g.Vs, l->stream));
  OVS_HIP(hipMemsetAsync(P_.GT, 0, sizeof(double2) * (size_t)cg * NF, l->stream));
  OVS_HIP(hipMemsetAsync(P_.GS, 0, sizeof(double2) * (size_t)cg * NF, l->stream));
  {
    std::vector<double2> ones((size_t)kLinTerms * nrhs, make_double2(1.0, 0.0));
    OVS_HIP(hipMemcpyAsync(coef_table(S, kTabOne), ones.data(), sizeof(double2) * ones.size(),
                           hipMemcpyHostToDevice, l->stream));
    std::vector<int> dints(2 + (size_t)nrhs);
    dints[0] = 0;
    dints[1] = nrhs;
    for (int r = 0; r < nrhs; ++r) dints[2 + r] = r;
    OVS_HIP(hipMemcpyAsync(P_.dints, dints.data(), sizeof(int) * dints.size(),
                           hipMemcpyHostToDevice, l->stream));
    if (md > 0)
      OVS_HIP(hipMemcpyAsync(coef_table(S2, kTabOne), ones.data(), sizeof(double2) * ones.size(),
                             hipMemcpyHostToDevice, l->stream));
    OVS_HIP(hipStreamSynchronize(l->stream));
  }
  launch_pack_f64((const double2*)b, B, nrhs, g, l->stream);
  launch_pack_f64((const double2*)chi, CHI, nrhs, g, l->stream);

  const Hop hA = make_hop(l->m_w, l->mu), hAd = make_hop(l->m_w, -l->mu);
  const Tuning tn = get_tuning(l, nrhs);
  auto applyA = [&](const double2* in, double2* out) {
    return launch_wilson(false, l->links, in, out, nrhs, g, hA, false, true, tn, l->stream);
  };
  auto applyAd = [&](const double2* in, double2* out) {
    return launch_wilson(false, l->links, in, out, nrhs, g, hAd, false, true, tn, l->stream);
  };
  // ta = A x and tb = A^dagger y in one launch (the dual stencil of the solve,
  // one thread per site for both operators): half the launches of a pair of
  // applications, and the links read once.  Every step of the forward pass,
  // its replay and the reverse sweep uses it, so replayed vectors stay
  // bitwise equal to the forward ones.
  auto applyBoth = [&](const double2* x, const double2* y, double2* ta, double2* tb) {
    DualArgs da{l->links, x, y, 0, false, P_.dints, ta, tb, P_.dpart2, P_.dints + 2,
                P_.dints + 1, nrhs, 0, 0, 0, 0, dual_tile};
    return launch_dual(false, da, g, hA, hAd, 1, l->stream);
  };
  auto mks = [&](const GradScalars& Sx, std::initializer_list<const double2*> xs, int tab,
                 double2* out, bool acc, std::initializer_list<const double2*> ys, int ndot,
                 double* part) {
    LinArgs la;
    int j = 0;
    for (const double2* p : xs) la.x[j++] = p;
    la.nterm = j;
    la.coef = coef_table(Sx, tab);
    la.out = out;
    la.accumulate = acc ? 1 : 0;
    j = 0;
    for (const double2* p : ys) {
      if (j < ndot) la.y[j] = p;
      ++j;
    }
    la.ndot = ndot;
    la.partials = part;
    return la;
  };
  auto mk = [&](std::initializer_list<const double2*> xs, int tab, double2* out, bool acc,
                std::initializer_list<const double2*> ys, int ndot, double* part) {
    return mks(S, xs, tab, out, acc, ys, ndot, part);
  };
  auto lin = [&](std::initializer_list<const double2*> xs, int tab, double2* out, bool acc,
                 std::initializer_list<const double2*> ys, int ndot, double* part) {
    launch_lin(mk(xs, tab, out, acc, ys, ndot, part), F, nrhs, l->stream);
  };
  auto lin2 = [&](std::initializer_list<const double2*> xs, int tab, double2* out, bool acc,
                  std::initializer_list<const double2*> ys, int ndot, double* part) {
    launch_lin(mks(S2, xs, tab, out, acc, ys, ndot, part), F, nrhs, l->stream);
  };
  // independent combinations (none reads another's output) in one launch
  auto multi = [&](std::initializer_list<LinArgs> las) {
    LinMulti m;
    for (const LinArgs& a : las) m.a[m.n++] = a;
    launch_lin_multi(m, F, nrhs, l->stream);
  };
  // a combination whose coefficients come from the scalar step run at the
  // start of the same launch (table `tab` of the step)
  auto from_step = [](LinArgs a, int tab) {
    a.tab = tab;
    return a;
  };
  auto step_of_s = [&](const GradScalars& Sx, int kind, int i, const double* pa, const double* pb,
                       bool global_tabs) {
    ScalarStep st;
    st.kind = kind;
    st.i = i;
    st.pa = pa;
    st.pb = pb;
    st.nchunk = nch;
    st.s = Sx;
    st.global_tabs = global_tabs ? 1 : 0;
    return st;
  };
  auto step_of = [&](int kind, int i, const double* pa, const double* pb, bool global_tabs) {
    return step_of_s(S, kind, i, pa, pb, global_tabs);
  };
  auto multi_step = [&](const ScalarStep& st, std::initializer_list<LinArgs> las) {
    LinMulti m;
    for (const LinArgs& a : las) m.a[m.n++] = a;
    launch_lin_multi_step(m, F, nrhs, st, l->stream);
  };
  auto copy = [&](double2* dst, const double2* src) {
    return hipMemcpyAsync(dst, src, sizeof(double2) * NF, hipMemcpyDeviceToDevice, l->stream);
  };
  // forward access: the whole basis, or a ring of three in the segment buffer
  auto Vf = [&](int i) { return store ? P_.V + (size_t)i * NF : P_.V + (size_t)(i % 3) * NF; };
  auto Wf = [&](int i) { return store ? P_.W + (size_t)i * NF : P_.W + (size_t)(i % 3) * NF; };
  // reverse access: the whole basis, or the current segment (indices base .. base + cseg + 1)
  int base = -1;
  auto Vr = [&](int i) { return store ? P_.V + (size_t)i * NF : P_.V + (size_t)(i - base) * NF; };
  auto Wr = [&](int i) { return store ? P_.W + (size_t)i * NF : P_.W + (size_t)(i - base) * NF; };
  // checkpoint j holds (v_{jc-1}, v_{jc}) and (w_{jc-1}, w_{jc}); v_{-1} = w_{-1} = 0
  auto save_ckpt = [&](int m) -> hipError_t {
    if (store || m % cseg) return hipSuccess;
    const int j = m / cseg;
    hipError_t e = copy(P_.ckV + (size_t)(2 * j + 1) * NF, Vf(m));
    if (e == hipSuccess) e = copy(P_.ckW + (size_t)(2 * j + 1) * NF, Wf(m));
    if (m > 0 && e == hipSuccess) e = copy(P_.ckV + (size_t)(2 * j) * NF, Vf(m - 1));
    if (m > 0 && e == hipSuccess) e = copy(P_.ckW + (size_t)(2 * j) * NF, Wf(m - 1));
    return e;
  };

  // ---- forward: v_1 = w_1 = b/|b| (deflated: v_1 = b_R/|b_R|, w_1 = b_L
  // |b_R| / conj(b_L^dagger b_R)), then the recurrences ----
  const ovs_deflation_s* d = defl;
  if (md > 0) {
    launch_defl(d->R, d->L, B, d->sgn, md, nrhs, F, P_.dpart, P_.CDb, P_.BR, P_.BL, P_.YEX,
                l->stream);
    // roles swapped: Q^dagger chi, Q chi and L S R^dagger chi; CDchi = (R^dag chi, L^dag chi)
    launch_defl(d->L, d->R, CHI, d->sgn, md, nrhs, F, P_.dpart, P_.CDchi, P_.CHIL, P_.CHIR,
                P_.YCHI, l->stream);
    lin({B}, kTabOne, nullptr, false, {nullptr}, 1, P[1]);
    lin({P_.BR}, kTabOne, nullptr, false, {nullptr, P_.BL}, 2, P[0]);
    launch_gf_start(S, P[0], P[1], nch, l->stream);
    lin({P_.BR}, kTabNorm, Vf(0), false, {CHI}, 1, P[3]);
    launch_gf_xbar(S, 0, P[3], nch, l->stream);
    lin({P_.BL}, kTabStartW, Wf(0), false, {}, 0, nullptr);
    if (y) OVS_HIP(copy(YA, P_.YEX));
  } else {
    lin({B}, kTabOne, nullptr, false, {nullptr}, 1, P[0]);
    launch_gf_norm(S, P[0], nch, l->stream);
    lin({B}, kTabNorm, Vf(0), false, {CHI}, 1, P[3]);
    launch_gf_xbar(S, 0, P[3], nch, l->stream);
    lin({B}, kTabNorm, Wf(0), false, {}, 0, nullptr);
  }
  OVS_HIP(save_ckpt(0));
  // Each step's scalar kernels (alpha, beta, xbar) run at the start of the
  // combination launch that follows them (launch_lin_step): five launches
  // per step.
  for (int i = 0; i < k; ++i) {
    if (i < k - 1) OVS_HIP(applyBoth(Vf(i), Wf(i), T, Sv));
    else OVS_HIP(applyA(Vf(i), T));
    // dots w_i^dagger t, |t|^2; xbar_i from the previous step's chi^dagger v_i
    if (i > 0)
      launch_lin_step(mk({T}, kTabOne, nullptr, false, {Wf(i), nullptr}, 2, P[0]), F, nrhs,
                      step_of(kStepXbar, i, P[3], nullptr, false), l->stream);
    else
      lin({T}, kTabOne, nullptr, false, {Wf(i), nullptr}, 2, P[0]);
    if (i == k - 1) {
      launch_gf_alpha(S, i, P[0], nch, l->stream);
      break;
    }
    // alpha_i (written by workgroup 0), then v~ and w~ in one launch (the dot
    // v~^dagger w~ reads v~ at the element the same thread has just written)
    const ScalarStep sa = step_of(kStepAlpha, i, P[0], nullptr, false);
    if (i > 0)
      multi_step(sa, {from_step(mk({T, Vf(i), Vf(i - 1)}, kTabV, Vf(i + 1), false, {nullptr}, 1,
                                   P[1]), kTabV),
                      from_step(mk({Sv, Wf(i), Wf(i - 1)}, kTabW, Wf(i + 1), false,
                                   {Vf(i + 1), nullptr}, 2, P[2]), kTabW)});
    else
      multi_step(sa, {from_step(mk({T, Vf(i)}, kTabV, Vf(i + 1), false, {nullptr}, 1, P[1]), kTabV),
                      from_step(mk({Sv, Wf(i)}, kTabW, Wf(i + 1), false, {Vf(i + 1), nullptr}, 2,
                                   P[2]), kTabW)});
    // beta_i, gamma_i, then the normalisation
    multi_step(step_of(kStepBeta, i, P[1], P[2], false),
               {from_step(mk({Vf(i + 1)}, kTabSV, Vf(i + 1), false, {CHI}, 1, P[3]), kTabSV),
                from_step(mk({Wf(i + 1)}, kTabSW, Wf(i + 1), false, {}, 0, nullptr), kTabSW)});
    OVS_HIP(save_ckpt(i + 1));
  }
  OVS_HIP(copy(TL, T));  // t_k = A v_k, needed by the first reverse step
  OVS_HIP(hipGetLastError());
  std::vector<int> status(nrhs);
  OVS_HIP(hipMemcpyAsync(status.data(), S.status, sizeof(int) * nrhs, hipMemcpyDeviceToHost,
                         l->stream));
  OVS_HIP(hipStreamSynchronize(l->stream));
  for (int r = 0; r < nrhs; ++r)
    if (status[r] != 0) return OVS_WARN_BREAKDOWN;  // the gradient needs k full iterations

  // ---- inner sign and its VJP ----
  rg.phase("inner_sign_vjp");
  ovs_status result = OVS_OK;
  for (int r = 0; r < nrhs; ++r) {
    const size_t rk = (size_t)r * k;
    std::vector<double2> prev, cur;
    // the first launch takes step kVjpHStart / 2 and forms the rule of step
    // kVjpHStart from the same solves (its even nodes): one launch for the
    // first comparison of two levels
    double h = 0.5 * kVjpHStart, change = 0.0;
    int lv = 0, used = 0;
    auto fetch_level = [&](const IsignVjpOut& o, std::vector<double2>& v) -> hipError_t {
      v.assign((size_t)3 * k, make_double2(0.0, 0.0));
      hipError_t e = hipMemcpyAsync(v.data(), o.x, sizeof(double2) * k, hipMemcpyDeviceToHost,
                                    l->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(v.data() + k, o.gd, sizeof(double2) * k, hipMemcpyDeviceToHost,
                           l->stream);
      if (e == hipSuccess && k > 1)
        e = hipMemcpyAsync(v.data() + 2 * k, o.gsup, sizeof(double2) * (k - 1),
                           hipMemcpyDeviceToHost, l->stream);
      return e;
    };
    for (bool first = true;; h *= 0.5, lv ^= 1, first = false) {
      int n0, nn;
      vjp_range(h, n0, nn);
      launch_isign_vjp(S.alpha + rk, S.beta + rk, S.gamma + rk, S.xbar + rk, k, h, n0, nn,
                       P_.vjp, P_.vo[lv], l->stream, first ? &P_.vo[1 - lv] : nullptr);
      OVS_HIP(hipGetLastError());
      OVS_HIP(fetch_level(P_.vo[lv], cur));
      if (first) OVS_HIP(fetch_level(P_.vo[1 - lv], prev));
      OVS_HIP(hipStreamSynchronize(l->stream));
      used = lv;
      if (!prev.empty()) {
        change = max_rel_change(cur, prev);
        if (change <= kVjpAccept) break;
      }
      if (h <= kVjpHMin) break;
      prev.swap(cur);
    }
    if (quad_err) quad_err[r] = change;
    if (change > 1e-6) result = OVS_WARN_SIGN_AMBIGUOUS;
    const IsignVjpOut& o = P_.vo[used];
    OVS_HIP(hipMemcpyAsync(S.x + rk, o.x, sizeof(double2) * k, hipMemcpyDeviceToDevice,
                           l->stream));
    OVS_HIP(hipMemcpyAsync(S.abar + rk, o.gd, sizeof(double2) * k, hipMemcpyDeviceToDevice,
                           l->stream));
    if (k > 1) {
      OVS_HIP(hipMemcpyAsync(S.bbar + rk, o.gsub_re, sizeof(double) * (k - 1),
                             hipMemcpyDeviceToDevice, l->stream));
      OVS_HIP(hipMemcpyAsync(S.gbar + rk, o.gsup, sizeof(double2) * (k - 1),
                             hipMemcpyDeviceToDevice, l->stream));
    }
  }

  // ---- deflated gradient: the coefficients of term (ii) and the forces of
  // term (iii) (see the head of this file) ----
  if (md > 0) {
    rg.phase("deflation_terms");
    const size_t nk = (size_t)nrhs * k;
    std::vector<cd> lam(md);
    std::vector<double> sg(md);
    for (int j = 0; j < md; ++j) {
      lam[j] = cd(d->lambda[2 * j], d->lambda[2 * j + 1]);
      sg[j] = d->lambda[2 * j] >= 0.0 ? 1.0 : -1.0;  // as the forward's sgn table
    }
    std::vector<double> cdb((size_t)md * nrhs * 4), cdchi((size_t)md * nrhs * 4);
    OVS_HIP(hipMemcpyAsync(cdb.data(), P_.CDb, sizeof(double) * cdb.size(), hipMemcpyDeviceToHost,
                           l->stream));
    OVS_HIP(hipMemcpyAsync(cdchi.data(), P_.CDchi, sizeof(double) * cdchi.size(),
                           hipMemcpyDeviceToHost, l->stream));
    auto cb = [&](int j, int r) {  // l_j^dagger b_r
      return cd(cdb[((size_t)j * nrhs + r) * 4], cdb[((size_t)j * nrhs + r) * 4 + 1]);
    };
    auto rchi = [&](int j, int r) {  // r_j^dagger chi_r
      return cd(cdchi[((size_t)j * nrhs + r) * 4], cdchi[((size_t)j * nrhs + r) * 4 + 1]);
    };
    // G_k of each source (host) from the run's coefficients
    struct Tri {
      std::vector<cd> d, lo, up, x;
      std::vector<double> nb;
    };
    auto fetch = [&](const GradScalars& Sx, Tri& t) -> hipError_t {
      std::vector<double2> a(nk), gm(nk), xx(nk);
      std::vector<double> bt(nk);
      t.nb.resize(nrhs);
      hipError_t e = hipMemcpyAsync(a.data(), Sx.alpha, sizeof(double2) * nk, hipMemcpyDeviceToHost, l->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(gm.data(), Sx.gamma, sizeof(double2) * nk, hipMemcpyDeviceToHost, l->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(xx.data(), Sx.x, sizeof(double2) * nk, hipMemcpyDeviceToHost, l->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(bt.data(), Sx.beta, sizeof(double) * nk, hipMemcpyDeviceToHost, l->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(t.nb.data(), Sx.nb, sizeof(double) * nrhs, hipMemcpyDeviceToHost, l->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(l->stream);
      t.d.resize(nk);
      t.lo.resize(nk);
      t.up.resize(nk);
      t.x.resize(nk);
      for (size_t q = 0; q < nk; ++q) {
        t.d[q] = cd(a[q].x, a[q].y);
        t.up[q] = cd(gm[q].x, gm[q].y);
        t.lo[q] = cd(bt[q], 0.0);
        t.x[q] = cd(xx[q].x, xx[q].y);
      }
      return e;
    };
    // z = (G_r - shift)^{-1} (x_r - s e_1)
    auto zsolve = [&](const Tri& t, int r, cd shift, double sj, std::vector<cd>& z) -> bool {
      const size_t rk = (size_t)r * k;
      z.assign(t.x.begin() + rk, t.x.begin() + rk + k);
      z[0] -= sj;
      return tri_solve(k, &t.d[rk], &t.lo[rk], &t.up[rk], shift, z);
    };
    Tri t1;
    OVS_HIP(fetch(S, t1));
    std::vector<double2> kap((size_t)k * nrhs * md);
    std::vector<cd> z(k);
    for (int r = 0; r < nrhs; ++r)
      for (int j = 0; j < md; ++j) {
        if (!zsolve(t1, r, lam[j], sg[j], z)) return OVS_WARN_BREAKDOWN;
        const cd a = rchi(j, r);
        for (int i = 0; i < k; ++i) {
          const cd v = std::conj(t1.nb[r] * z[i]) * a;
          kap[((size_t)i * nrhs + r) * md + j] = make_double2(v.real(), v.imag());
        }
      }
    OVS_HIP(hipMemcpyAsync(P_.kappa, kap.data(), sizeof(double2) * kap.size(),
                           hipMemcpyHostToDevice, l->stream));

    // second run: A^dagger from Q^dagger chi, left start Q chi, full basis kept
    auto V2 = [&](int i) { return P_.V2 + (size_t)i * NF; };
    auto W2 = [&](int i) { return P_.W2 + (size_t)(i % 3) * NF; };
    lin2({CHI}, kTabOne, nullptr, false, {nullptr}, 1, P[1]);
    lin2({P_.CHIL}, kTabOne, nullptr, false, {nullptr, P_.CHIR}, 2, P[0]);
    launch_gf_start(S2, P[0], P[1], nch, l->stream);
    lin2({P_.CHIL}, kTabNorm, V2(0), false, {}, 0, nullptr);
    lin2({P_.CHIR}, kTabStartW, W2(0), false, {}, 0, nullptr);
    // the same launches per step as the main forward pass: the operator pair
    // in one dual-stencil launch (here t = A^dagger v, s = A w), alpha and
    // beta at the start of the combinations that use them
    for (int i = 0; i < k; ++i) {
      if (i < k - 1) OVS_HIP(applyBoth(W2(i), V2(i), Sv, T));
      else OVS_HIP(applyAd(V2(i), T));
      lin2({T}, kTabOne, nullptr, false, {W2(i), nullptr}, 2, P[0]);
      if (i == k - 1) {
        launch_gf_alpha(S2, i, P[0], nch, l->stream);
        break;
      }
      const ScalarStep sa = step_of_s(S2, kStepAlpha, i, P[0], nullptr, false);
      if (i > 0)
        multi_step(sa, {from_step(mks(S2, {T, V2(i), V2(i - 1)}, kTabV, V2(i + 1), false, {nullptr},
                                      1, P[1]), kTabV),
                        from_step(mks(S2, {Sv, W2(i), W2(i - 1)}, kTabW, W2(i + 1), false,
                                      {V2(i + 1), nullptr}, 2, P[2]), kTabW)});
      else
        multi_step(sa, {from_step(mks(S2, {T, V2(i)}, kTabV, V2(i + 1), false, {nullptr}, 1, P[1]),
                                  kTabV),
                        from_step(mks(S2, {Sv, W2(i)}, kTabW, W2(i + 1), false,
                                      {V2(i + 1), nullptr}, 2, P[2]), kTabW)});
      multi_step(step_of_s(S2, kStepBeta, i, P[1], P[2], false),
                 {from_step(mks(S2, {V2(i + 1)}, kTabSV, V2(i + 1), false, {}, 0, nullptr), kTabSV),
                  from_step(mks(S2, {W2(i + 1)}, kTabSW, W2(i + 1), false, {}, 0, nullptr),
                            kTabSW)});
    }
    OVS_HIP(hipGetLastError());
    OVS_HIP(hipMemcpyAsync(status.data(), S2.status, sizeof(int) * nrhs, hipMemcpyDeviceToHost,
                           l->stream));
    OVS_HIP(hipStreamSynchronize(l->stream));
    for (int r = 0; r < nrhs; ++r)
      if (status[r] != 0) return OVS_WARN_BREAKDOWN;
    // x' = sgn(G') e_1 by the same quadrature (zero adjoint seed)
    for (int r = 0; r < nrhs; ++r) {
      const size_t rk = (size_t)r * k;
      std::vector<double2> prev, cur;
      double h = 0.5 * kVjpHStart, change = 0.0;  // first launch: two levels, as above
      int lv = 0, used = 0;
      for (bool first = true;; h *= 0.5, lv ^= 1, first = false) {
        int n0, nn;
        vjp_range(h, n0, nn);
        launch_isign_vjp(S2.alpha + rk, S2.beta + rk, S2.gamma + rk, S2.xbar + rk, k, h, n0, nn,
                         P_.vjp, P_.vo[lv], l->stream, first ? &P_.vo[1 - lv] : nullptr);
        OVS_HIP(hipGetLastError());
        cur.assign(k, make_double2(0.0, 0.0));
        OVS_HIP(hipMemcpyAsync(cur.data(), P_.vo[lv].x, sizeof(double2) * k,
                               hipMemcpyDeviceToHost, l->stream));
        if (first) {
          prev.assign(k, make_double2(0.0, 0.0));
          OVS_HIP(hipMemcpyAsync(prev.data(), P_.vo[1 - lv].x, sizeof(double2) * k,
                                 hipMemcpyDeviceToHost, l->stream));
        }
        OVS_HIP(hipStreamSynchronize(l->stream));
        used = lv;
        if (!prev.empty()) {
          change = max_rel_change(cur, prev);
          if (change <= kVjpAccept) break;
        }
        if (h <= kVjpHMin) break;
        prev.swap(cur);
      }
      if (change > 1e-6) result = OVS_WARN_SIGN_AMBIGUOUS;
      OVS_HIP(hipMemcpyAsync(S2.x + rk, P_.vo[used].x, sizeof(double2) * k,
                             hipMemcpyDeviceToDevice, l->stream));
    }
    Tri t2;
    OVS_HIP(fetch(S2, t2));
    std::vector<double2> cq((size_t)md * k * nrhs), cl((size_t)md * md, make_double2(0.0, 0.0));
    for (int j = 0; j < md; ++j) {
      for (int r = 0; r < nrhs; ++r) {
        if (!zsolve(t2, r, std::conj(lam[j]), sg[j], z)) return OVS_WARN_BREAKDOWN;
        const cd w = std::conj(cb(j, r)) * t2.nb[r];
        for (int i = 0; i < k; ++i) {
          const cd v = w * z[i];
          cq[(size_t)j * k * nrhs + (size_t)i * nrhs + r] = make_double2(v.real(), v.imag());
        }
      }
      for (int q = 0; q < md; ++q) {
        if (q == j || sg[q] == sg[j]) continue;
        cd v = 0.0;
        for (int r = 0; r < nrhs; ++r) v += std::conj(cb(j, r)) * rchi(q, r);
        v *= (sg[q] - sg[j]) / (std::conj(lam[q]) - std::conj(lam[j]));
        cl[(size_t)j * md + q] = make_double2(v.real(), v.imag());
      }
    }
    const int ku[2] = {k * nrhs, md};
    OVS_HIP(hipMemcpyAsync(P_.coefQ, cq.data(), sizeof(double2) * cq.size(), hipMemcpyHostToDevice,
                           l->stream));
    OVS_HIP(hipMemcpyAsync(P_.coefL, cl.data(), sizeof(double2) * cl.size(), hipMemcpyHostToDevice,
                           l->stream));
    OVS_HIP(hipMemcpyAsync(P_.kused, ku, sizeof(ku), hipMemcpyHostToDevice, l->stream));
    // Q_j = sum_r conj(c_jr) q_jr, force Re <Q_j, dA r_j>
    for (int j = 0; j < md; ++j) {
      launch_combine(false, P_.V2, F, F, P_.coefQ + (size_t)j * k * nrhs, k * nrhs, P_.kused,
                     nullptr, P_.QJ, 1, l->stream);
      launch_combine(false, d->L, F, F, P_.coefL + (size_t)j * md, md, P_.kused + 1, P_.QJ, P_.QJ,
                     1, l->stream);
      launch_gforce(P_.Fg, P_.QJ, d->R + (size_t)j * F, nullptr, nullptr, F, 1, g, hA, hAd,
                    l->stream);
    }
    OVS_HIP(hipGetLastError());
    OVS_HIP(hipStreamSynchronize(l->stream));  // host coefficient vectors are released
  }
  // forces of the sweep: Q^dagger tbar (+ the term (ii) vector of step i) and Q sbar
  auto ptb = [&](int i, const double2* tb, double2* out) -> const double2* {
    if (md == 0) return tb;
    launch_defl_proj(d->R, d->L, tb, md, nrhs, F, P_.dpart, P_.CDt,
                     P_.kappa + (size_t)i * nrhs * md, nullptr, out, l->stream);
    return out;
  };
  auto psb = [&](const double2* sb, double2* out) -> const double2* {
    if (md == 0) return sb;
    launch_defl_proj(d->R, d->L, sb, md, nrhs, F, P_.dpart, P_.CDt, nullptr, out, nullptr,
                     l->stream);
    return out;
  };
  // force-group slots of step i; without deflation tbar_i and sbar_i are
  // formed there directly (sbar_{i+1} of the previous step is in the next
  // slot), with deflation their projections go there
  auto slotT = [&](int i) { return P_.GT + (size_t)(i % cg) * NF; };
  auto slotS = [&](int i) { return P_.GS + (size_t)(i % cg) * NF; };
  auto TBc = [&](int i) { return md == 0 ? slotT(i) : TB; };
  auto WTBc = [&](int i) { return md == 0 ? slotS(i) : WTB[i & 1]; };

  // ---- reverse sweep, segment by segment from the last ----
  rg.phase("reverse_sweep");
  for (int j = nseg - 1; j >= 0; --j) {
    const int lo = j * cseg, hi = std::min((j + 1) * cseg, k) - 1;
    if (!store) {
      // replay v_{lo+1} .. v_{top} from the checkpoint, as in the forward pass
      base = lo - 1;
      const int top = std::min((j + 1) * cseg, k - 1);
      OVS_HIP(copy(Vr(lo - 1), P_.ckV + (size_t)(2 * j) * NF));
      OVS_HIP(copy(Vr(lo), P_.ckV + (size_t)(2 * j + 1) * NF));
      OVS_HIP(copy(Wr(lo - 1), P_.ckW + (size_t)(2 * j) * NF));
      OVS_HIP(copy(Wr(lo), P_.ckW + (size_t)(2 * j + 1) * NF));
      for (int i = lo; i < top; ++i) {
        // the rows of step i from the stored coefficients, formed in each launch
        // and v~, w~ and their normalisation in one launch (the scaling reads
        // each element the same thread has just written)
        const ScalarStep sc = step_of(kStepCoef, i, nullptr, nullptr, false);
        OVS_HIP(applyBoth(Vr(i), Wr(i), T, Sv));
        const LinArgs nv =
            from_step(mk({Vr(i + 1)}, kTabSV, Vr(i + 1), false, {}, 0, nullptr), kTabSV);
        const LinArgs nw =
            from_step(mk({Wr(i + 1)}, kTabSW, Wr(i + 1), false, {}, 0, nullptr), kTabSW);
        if (i > 0)
          multi_step(sc, {from_step(mk({T, Vr(i), Vr(i - 1)}, kTabV, Vr(i + 1), false, {}, 0,
                                       nullptr), kTabV),
                          from_step(mk({Sv, Wr(i), Wr(i - 1)}, kTabW, Wr(i + 1), false, {}, 0,
                                       nullptr), kTabW),
                          nv, nw});
        else
          multi_step(sc, {from_step(mk({T, Vr(i)}, kTabV, Vr(i + 1), false, {}, 0, nullptr), kTabV),
                          from_step(mk({Sv, Wr(i)}, kTabW, Wr(i + 1), false, {}, 0, nullptr),
                                    kTabW),
                          nv, nw});
      }
    }
    for (int i = hi; i >= lo; --i) {
      if (i == k - 1) {
        const int c = i & 1;
        launch_gr_first(S, l->stream);
        LinMulti m0;
        m0.a[m0.n++] = mk({Wr(i)}, kTabSV, TB, false, {}, 0, nullptr);    // tbar
        m0.a[m0.n++] = mk({CHI}, kTabSW, VB[c], false, {}, 0, nullptr);   // vbar (direct part)
        m0.a[m0.n++] = mk({TL}, kTabWB, WB[c], false, {Wr(i)}, 1, P[3]);  // wbar, complete
        if (y) m0.a[m0.n++] = mk({Vr(i)}, kTabY, YA, true, {}, 0, nullptr);
        launch_lin_multi(m0, F, nrhs, l->stream);
        OVS_HIP(applyAd(TB, T1));
        lin({T1}, kTabOne, VB[c], true, {Vr(i)}, 1, P[2]);    // vbar += A^dag tbar
        launch_gforce(P_.Fg, ptb(i, TB, P_.TBp), Vr(i), nullptr, nullptr, F, nrhs, g, hA, hAd,
                      l->stream);
        continue;
      }
      const int c = i & 1, p = (i + 1) & 1;
      // step 1 of the reverse scalars (from the dots of vbar_{i+1}, wbar_{i+1})
      const ScalarStep s1 = step_of(kStepS1, i, P[2], P[3], false);
      double2* const tbi = TBc(i);
      double2* const sbi = WTBc(i);
      const double2* const sbn = WTBc(i + 1);  // sbar_{i+1}
      if (i > 0)
        multi_step(s1, {from_step(mk({VB[p], Vr(i + 1), Wr(i + 1)}, kTabV, VTB[c], false,
                                     {Vr(i), Vr(i - 1)}, 2, P[0]), kTabV),
                        from_step(mk({WB[p], Vr(i + 1)}, kTabW, sbi, false,
                                     {Wr(i), Wr(i - 1)}, 2, P[1]), kTabW)});
      else
        multi_step(s1, {from_step(mk({VB[p], Vr(i + 1), Wr(i + 1)}, kTabV, VTB[c], false, {Vr(i)},
                                     1, P[0]), kTabV),
                        from_step(mk({WB[p], Vr(i + 1)}, kTabW, sbi, false, {Wr(i)}, 1, P[1]),
                                  kTabW)});
      // step 2 (abar_i; bbar_{i-1}, gbar_{i-1} written by workgroup 0)
      LinMulti m2;
      m2.a[m2.n++] = from_step(mk({VTB[c], Wr(i)}, kTabSV, tbi, false, {}, 0, nullptr), kTabSV);
      m2.a[m2.n++] = from_step(mk({CHI, VTB[p], VTB[c]}, kTabSW, VB[c], false, {}, 0, nullptr),
                               kTabSW);
      if (i > 0)
        m2.a[m2.n++] = from_step(mk({sbn, sbi, Vr(i + 1), Vr(i), Vr(i - 1)}, kTabWB, WB[c], false,
                                    {}, 0, nullptr), kTabWB);
      else
        m2.a[m2.n++] = from_step(mk({sbn, sbi, Vr(i + 1), Vr(i)}, kTabWB, WB[c], false, {}, 0,
                                    nullptr), kTabWB);
      if (y) m2.a[m2.n++] = from_step(mk({Vr(i)}, kTabY, YA, true, {}, 0, nullptr), kTabY);
      launch_lin_multi_step(m2, F, nrhs, step_of(kStepS2, i, P[0], P[1], false), l->stream);
      OVS_HIP(applyBoth(sbi, tbi, T2, T1));
      multi({mk({T1}, kTabOne, VB[c], true, {Vr(i)}, 1, P[2]),
             mk({T2}, kTabOne, WB[c], true, {Wr(i)}, 1, P[3])});
      // the force of this step waits in its group's slots; a group (the steps
      // i .. i + cg - 1 below k - 1) is summed when its lowest step is done
      if (md > 0) {
        ptb(i, tbi, slotT(i));
        psb(sbi, slotS(i));
      }
      if (i % cg == 0) {
        const int n = std::min(i + cg - 1, k - 2) - i + 1;
        launch_gforce_group(P_.Fg, slotT(i), Vr(i), slotS(i), Wr(i), n, NF, F, nrhs, g, hA, hAd,
                            l->stream);
      }
    }
  }
  if (md > 0) {
    // bbar_R, bbar_L from vbar_1, wbar_1, then grad_b = Q^dagger bbar_R + Q bbar_L
    // + L S R^dagger chi  (segment 0 holds v_1, w_1)
    lin({VB[0]}, kTabOne, nullptr, false, {Vr(0)}, 1, P[0]);
    lin({WB[0]}, kTabOne, nullptr, false, {Wr(0)}, 1, P[1]);
    launch_gr_final_defl(S, P[0], P[1], nch, l->stream);
    lin({VB[0], P_.BL, P_.BR}, kTabFin, T1, false, {}, 0, nullptr);
    lin({WB[0], P_.BR}, kTabFinW, T2, false, {}, 0, nullptr);
    launch_defl_proj(d->R, d->L, T1, md, nrhs, F, P_.dpart, P_.CDt, nullptr, nullptr, GB,
                     l->stream);
    launch_defl_proj(d->R, d->L, T2, md, nrhs, F, P_.dpart, P_.CDt, nullptr, T2, nullptr,
                     l->stream);
    lin({T2, P_.YCHI}, kTabOne, GB, true, {}, 0, nullptr);
  } else {
    // grad_b = ubar/|b| + nbar v_1,  ubar = vbar_1 + wbar_1  (segment 0 holds v_1)
    lin({VB[0], WB[0]}, kTabOne, T1, false, {Vr(0)}, 1, P[0]);
    launch_gr_final(S, P[0], nch, l->stream);
    lin({T1, Vr(0)}, kTabFin, GB, false, {}, 0, nullptr);
  }
  launch_unpack_f64(GB, (double2*)grad_b, nrhs, g, l->stream);
  launch_gforce_out(P_.Fg, (const double2*)l->links, g, l->bc, (double2*)grad_U, P_.fparts,
                    P_.gmu, l->stream);
  if (y) launch_unpack_f64(YA, (double2*)y, nrhs, g, l->stream);
  OVS_HIP(hipGetLastError());
  OVS_HIP(hipMemcpyAsync(grad_mu, P_.gmu, sizeof(double), hipMemcpyDeviceToHost, l->stream));
  OVS_HIP(hipStreamSynchronize(l->stream));
  return result;
}

extern "C" ovs_status ovs_link_force(ovs_lattice l, const void* U, const void* grad_U, void* force) {
  if (!l || !U || !grad_U || !force || l->parent) return OVS_ERR_ARG;
  StreamScope sc(l);
  launch_link_force((const double2*)U, (const double2*)grad_U, (double2*)force, 4L * l->g.V,
                    l->stream);
  OVS_HIP(hipGetLastError());
  return OVS_OK;
}

extern "C" ovs_status ovs_sign_apply_vjp(ovs_lattice l, ovs_deflation defl, int32_t n_defl,
                                         const void* b, const void* chi, int32_t nrhs, int32_t k,
                                         int32_t flags, void* y, void* grad_b, double* grad_mu,
                                         void* grad_U, double* quad_err, void* workspace,
                                         size_t ws_bytes) {
  return vjp_impl(l, defl, n_defl, b, chi, nrhs, k, flags, y, grad_b, grad_mu, grad_U, quad_err,
                  workspace, workspace ? ws_bytes : 0, nullptr);
}

extern "C" ovs_status ovs_vjp_workspace_size(ovs_lattice l, ovs_deflation defl, int32_t n_defl,
                                             int32_t nrhs, int32_t k, int32_t flags,
                                             size_t* bytes) {
  if (!bytes) return OVS_ERR_ARG;
  *bytes = 0;
  return vjp_impl(l, defl, n_defl, nullptr, nullptr, nrhs, k, flags, nullptr, nullptr, nullptr,
                  nullptr, nullptr, nullptr, 0, bytes);
}
