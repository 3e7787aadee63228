#pragma once
// V-cycle on the device (section 2, "AMG solve"): the per-level storage and
// the driver that launches the fused SpMV kernels of one cycle.
//
// Per level l < L (zero initial guess on every level; one pre- and one
// post-sweep of the diagonal smoother m in the common configuration):
//   r_l     = f_l - A_l (m .* f_l)      pre-sweep fused into the residual
//                                       (level 1: (A_1 diag(m)) f_1, stored once)
//   f_{l+1} = R_l r_l                   restriction (also m .* f_{l+1})
//   ... coarser levels, then z_L = A_L^-1 f_L (dense inverse, FP64) ...
//   y_l     = m .* f_l + P_l z_{l+1}    prolongation + correction, pre-sweep recomputed
//   z_l     = y_l + m .* (f_l - A_l y_l)  post-sweep (level 1 of PCG also forms r . z)
// Chebyshev sweeps replace the two smoothing steps (chebyshev.hpp).

#include <hip/hip_runtime.h>

#include <type_traits>
#include <vector>

#include "chebyshev.hpp"
#include "device.hpp"
#include "tail.hpp"

namespace amg {

template <class T>
struct DevLevel {
  int32_t n = 0, nc = 0;
  DevCsr<T> A, P, R;
  DevCsr<T> As;  // level 1: A diag(m), same pattern as A (its own values)
  T* m = nullptr;
  T* f = nullptr;  // right-hand side (unused on level 0: the caller's vector)
  T* r = nullptr;  // residual
  T* y = nullptr;  // prolongated correction
  T* t = nullptr;  // ping-pong buffer for repeated sweeps
  T* zp[2] = {nullptr, nullptr};  // stored pre-smoothed iterate (npre > 1)
  T* z = nullptr;   // output on levels > 0
  T* mf = nullptr;  // m .* f, written by the restriction (levels > 0, npre = 1);
                    // Chebyshev: the first direction (m .* f) / theta
  T* dc[2] = {nullptr, nullptr};  // Chebyshev directions (ping-pong)
  ChebCoef<T> cheb;               // Chebyshev coefficients
};

template <class T>
struct DevHierarchy {
  std::vector<DevLevel<T>> lev;  // levels 0 .. L-2
  T* fL = nullptr;               // coarsest right-hand side / solution
  T* zL = nullptr;
  // Fused coarse tail: levels tail_first .. L-2 and the coarse solve in one
  // launch of tail_grid workgroups (tail_first = 0: not fused).
  int tail_first = 0;
  int tail_grid = 0;
  TailSync* tail_sync = nullptr;
  uint64_t tail_limit = 0;
};

struct VcycleOpts {
  int npre = 1, npost = 1;
  int relax = AMG_SPAI0;
};

// ------------------------------------------------------------------ V-cycle

template <class T>
class Vcycle {
 public:
  Vcycle(DevHierarchy<T>* h, const double* Ainv, int32_t nL, VcycleOpts o)
      : h_(h), Ainv_(Ainv), nL_(nL), o_(o) {}

  // z0 = V(f0); f0, z0 double[n].  With DOT, writes the partials of f0 . z0
  // and returns their count; otherwise returns 0.
  template <int DOT>
  int run(const double* f0, double* z0, double* partials, const int* skip, hipStream_t s) {
    const int L = static_cast<int>(h_->lev.size()) + 1;
    if (L == 1) {
      coarse_gemv_kernel<double, double><<<nL_, kBS, 0, s>>>(nL_, Ainv_, f0, z0, skip);
      AMG_LAUNCHED();
      if (DOT) {
        int nb = vec_blocks(nL_);
        dot_kernel<<<nb, kVecBS, 0, s>>>(nL_, f0, z0, partials, skip);
        AMG_LAUNCHED();
        return nb;
      }
      return 0;
    }
    // levels >= tail run fused in one launch (with the coarse solve)
    const int tail = use_tail() ? h_->tail_first : L - 1;
    // down
    for (int l = 0; l < tail; ++l) {
      DevLevel<T>& lv = h_->lev[l];
      DevLevel<T>* next = (l + 1 < L - 1) ? &h_->lev[l + 1] : nullptr;
      if (l == 0) down<double>(lv, f0, next, skip, s);
      else down<T>(lv, lv.f, next, skip, s);
    }
    if (tail < L - 1) {
      launch_tail(tail, skip, s);
    } else {
      coarse_gemv_kernel<T, T><<<nL_, kBS, 0, s>>>(nL_, Ainv_, h_->fL, h_->zL, skip);
      AMG_LAUNCHED();
    }
    // up
    int nparts = 0;
    for (int l = tail - 1; l >= 0; --l) {
      DevLevel<T>& lv = h_->lev[l];
      const T* zc = (l + 1 < L - 1) ? h_->lev[l + 1].z : h_->zL;
      if (l == 0) nparts = up<double, double, DOT>(lv, f0, zc, z0, partials, skip, s);
      else up<T, T, 0>(lv, lv.f, zc, lv.z, partials, skip, s);
    }
    return nparts;
  }

 private:
  // Pre-relaxation, residual and restriction of one level.  `next` is the
  // next level (NULL when that is the coarsest).  On levels > 0 with one
  // pre-sweep, m .* f was written by the restriction that produced f.
  template <class TF>
  void down(DevLevel<T>& lv, const TF* f, DevLevel<T>* next, const int* skip, hipStream_t s) {
    if (o_.relax == AMG_CHEBYSHEV && o_.npre > 0) {
      cheb_down(lv, f, next, skip, s);
      return;
    }
    T* fnext = next ? next->f : h_->fL;
    auto restrict_from = [&](auto gather) {
      if (next && o_.npre == 1)
        launch_spmv(lv.R, gather, EpiRestrict<T>{next->f, next->mf, next->m}, nullptr, skip, s);
      else
        launch_spmv(lv.R, gather, EpiStore<T, T>{fnext}, nullptr, skip, s);
    };
    if (o_.npre == 0) {
      restrict_from(GatherX<T, TF>{f});
      return;
    }
    if (o_.npre == 1) {
      if (lv.As.val) {
        // r = f - (A diag(m)) f: one gathered vector instead of m and f
        launch_spmv(lv.As, GatherX<T, TF>{f}, EpiResid<T, TF>{lv.r, f}, nullptr, skip, s);
      } else if constexpr (std::is_same<TF, T>::value) {
        if (lv.mf) {
          launch_spmv(lv.A, GatherX<T, T>{lv.mf}, EpiResid<T, TF>{lv.r, f}, nullptr, skip, s);
        } else {
          launch_spmv(lv.A, GatherMF<T, TF>{lv.m, f}, EpiResid<T, TF>{lv.r, f}, nullptr, skip, s);
        }
      } else {
        launch_spmv(lv.A, GatherMF<T, TF>{lv.m, f}, EpiResid<T, TF>{lv.r, f}, nullptr, skip, s);
      }
    } else {
      scale_kernel<T, TF><<<vec_blocks(lv.n), kVecBS, 0, s>>>(lv.n, lv.zp[0], lv.m, f, skip);
      AMG_LAUNCHED();
      int cur = 0;
      for (int k = 1; k < o_.npre; ++k) {
        launch_spmv(lv.A, GatherX<T, T>{lv.zp[cur]}, EpiSmooth<T, TF, T, 0>{lv.zp[1 - cur], lv.zp[cur], lv.m, f},
                    nullptr, skip, s);
        cur = 1 - cur;
      }
      pre_cur_ = cur;
      launch_spmv(lv.A, GatherX<T, T>{lv.zp[cur]}, EpiResid<T, TF>{lv.r, f}, nullptr, skip, s);
    }
    restrict_from(GatherX<T, T>{lv.r});
  }

  // Prolongation + correction and post-relaxation of one level; output zout.
  template <class TF, class TZ, int DOT>
  int up(DevLevel<T>& lv, const TF* f, const T* zc, TZ* zout, double* partials, const int* skip,
         hipStream_t s) {
    if (o_.relax == AMG_CHEBYSHEV) return cheb_up<TF, TZ, DOT>(lv, f, zc, zout, partials, skip, s);
    if (o_.npre == 0) {
      launch_spmv(lv.P, GatherX<T, T>{zc}, EpiProlong<T, TF, 0>{lv.y, lv.m, f, nullptr}, nullptr, skip, s);
    } else if (o_.npre == 1) {
      if (lv.mf)
        launch_spmv(lv.P, GatherX<T, T>{zc}, EpiProlong<T, TF, 2>{lv.y, lv.m, f, lv.mf}, nullptr, skip, s);
      else
        launch_spmv(lv.P, GatherX<T, T>{zc}, EpiProlong<T, TF, 1>{lv.y, lv.m, f, nullptr}, nullptr, skip, s);
    } else {
      launch_spmv(lv.P, GatherX<T, T>{zc}, EpiProlong<T, TF, 2>{lv.y, lv.m, f, lv.zp[pre_cur_]}, nullptr,
                  skip, s);
    }
    if (o_.npost == 0) {
      int nb = vec_blocks(lv.n);
      copy_dot_kernel<T, TF, TZ, DOT><<<nb, kVecBS, 0, s>>>(lv.n, zout, lv.y, f, partials, skip);
      AMG_LAUNCHED();
      return DOT ? nb : 0;
    }
    T* cur = lv.y;
    T* other = lv.t;
    int nparts = 0;
    for (int k = 0; k < o_.npost; ++k) {
      const bool last = (k == o_.npost - 1);
      if (last) {
        nparts = launch_spmv(lv.A, GatherX<T, T>{cur}, EpiSmooth<T, TF, TZ, DOT>{zout, cur, lv.m, f}, partials,
                             skip, s);
      } else {
        launch_spmv(lv.A, GatherX<T, T>{cur}, EpiSmooth<T, TF, T, 0>{other, cur, lv.m, f}, nullptr, skip, s);
        std::swap(cur, other);
      }
    }
    return DOT ? nparts : 0;
  }

  // ---- Chebyshev relaxation (one sweep = `degree` steps, see chebyshev.hpp)

  // Pre-sweeps from a zero guess, x in zp[]; the last one keeps its residual
  // in lv.r, which is restricted.
  template <class TF>
  void cheb_down(DevLevel<T>& lv, const TF* f, DevLevel<T>* next, const int* skip, hipStream_t s) {
    int xi = 0;
    for (int k = 0; k < o_.npre; ++k) {
      const bool keep_r = (k == o_.npre - 1);
      xi = cheb_sweep<TF, T, 0>(lv, f, k == 0, keep_r, xi, lv.zp, lv.zp[xi], nullptr, skip, s);
    }
    pre_cur_ = xi;
    if (next)
      launch_spmv(lv.R, GatherX<T, T>{lv.r}, EpiRestrictCheb<T>{next->f, next->mf, next->m, next->cheb.theta},
                  nullptr, skip, s);
    else
      launch_spmv(lv.R, GatherX<T, T>{lv.r}, EpiStore<T, T>{h_->fL}, nullptr, skip, s);
  }

  // Prolongation + correction, then post-sweeps from y; the last writes zout.
  template <class TF, class TZ, int DOT>
  int cheb_up(DevLevel<T>& lv, const TF* f, const T* zc, TZ* zout, double* partials, const int* skip,
              hipStream_t s) {
    if (o_.npre == 0)
      launch_spmv(lv.P, GatherX<T, T>{zc}, EpiProlong<T, TF, 0>{lv.y, lv.m, f, nullptr}, nullptr, skip, s);
    else
      launch_spmv(lv.P, GatherX<T, T>{zc}, EpiProlong<T, TF, 2>{lv.y, lv.m, f, lv.zp[pre_cur_]}, nullptr,
                  skip, s);
    if (o_.npost == 0) {
      int nb = vec_blocks(lv.n);
      copy_dot_kernel<T, TF, TZ, DOT><<<nb, kVecBS, 0, s>>>(lv.n, zout, lv.y, f, partials, skip);
      AMG_LAUNCHED();
      return DOT ? nb : 0;
    }
    T* xs[2] = {lv.y, lv.t};
    int xi = 0;
    for (int k = 0; k + 1 < o_.npost; ++k) xi = cheb_sweep<TF, T, 0>(lv, f, false, false, xi, xs, xs[xi], nullptr, skip, s);
    cheb_nparts_ = 0;
    cheb_sweep<TF, TZ, DOT>(lv, f, false, false, xi, xs, zout, partials, skip, s);
    return DOT ? cheb_nparts_ : 0;
  }

  // One step (s = A d) of a sweep; coefficients of step j.
  template <int Z, int D0, int MODE, int DOT, class TF, class TZ>
  int cheb_step(DevLevel<T>& lv, const TF* f, const T* d, T* dn, T* x, TZ* out, int j, double* partials,
                const int* skip, hipStream_t s) {
    const ChebCoef<T>& c = lv.cheb;
    EpiChebStep<T, TF, TZ, Z, D0, MODE, DOT> e{x, lv.r, d, dn, lv.m, f, c.theta, c.c1[j], c.c2[j], out};
    if constexpr (Z && !D0)
      return launch_spmv(lv.A, GatherMFc<T, TF>{lv.m, f, c.theta}, e, DOT ? partials : nullptr, skip, s);
    else
      return launch_spmv(lv.A, GatherX<T, T>{d}, e, DOT ? partials : nullptr, skip, s);
  }

  // One sweep on level lv for A x = f with x = xs[xi] (ignored when
  // from_zero).  keep_r: the last step is carried out in full, leaving the
  // result in xs[xi] and its residual in lv.r.  Otherwise the result goes to
  // out (which may be xs[xi] except when the sweep is a single step from a
  // nonzero guess: that product gathers x, so the result goes to
  // xs[1 - xi]).  Returns the index of the buffer holding the result when out
  // is one of xs; DOT partial counts go to cheb_nparts_.
  template <class TF, class TZ, int DOT>
  int cheb_sweep(DevLevel<T>& lv, const TF* f, bool from_zero, bool keep_r, int xi, T* const* xs, TZ* out,
                 double* partials, const int* skip, hipStream_t s) {
    const ChebCoef<T>& c = lv.cheb;
    const int k = c.degree;
    T* x = xs[xi];
    const T* d0 = lv.mf;  // stored first direction (levels > 0), else recomputed
    if (from_zero && k == 1 && !keep_r) {
      // x = d0 and no residual wanted: no product.  (Never the DOT sweep,
      // which starts from the prolongated iterate.)
      if (d0)
        cheb_first_kernel<T, TF, TZ, 1><<<vec_blocks(lv.n), kVecBS, 0, s>>>(lv.n, out, d0, lv.m, f, c.theta, skip);
      else
        cheb_first_kernel<T, TF, TZ, 0><<<vec_blocks(lv.n), kVecBS, 0, s>>>(lv.n, out, d0, lv.m, f, c.theta, skip);
      AMG_LAUNCHED();
      return xi;
    }
    int cur = 0;
    if (!from_zero) {
      if (k == 1 && !keep_r) {
        TZ* o = out;
        int res = xi;
        if (static_cast<const void*>(out) == static_cast<const void*>(x)) {
          o = reinterpret_cast<TZ*>(xs[1 - xi]);
          res = 1 - xi;
        }
        int nb = launch_spmv(lv.A, GatherX<T, T>{x},
                             EpiChebInit<T, TF, TZ, 1, DOT>{x, lv.r, nullptr, lv.m, f, c.theta, o},
                             DOT ? partials : nullptr, skip, s);
        if (DOT) cheb_nparts_ = nb;
        return res;
      }
      launch_spmv(lv.A, GatherX<T, T>{x}, EpiChebInit<T, TF, T, 0, 0>{x, lv.r, lv.dc[0], lv.m, f, c.theta, nullptr},
                  nullptr, skip, s);
    }
    for (int j = 0; j < k; ++j) {
      const bool zero = from_zero && j == 0;
      const int mode = (j == k - 1) ? kChebLast : (!keep_r && j == k - 2) ? kChebFused : kChebMid;
      const T* dcur = zero ? d0 : lv.dc[cur];
      T* dnext = zero ? lv.dc[0] : lv.dc[1 - cur];
      if (mode == kChebFused) {
        int nb;
        if (!zero) nb = cheb_step<0, 0, kChebFused, DOT>(lv, f, dcur, dnext, x, out, j, partials, skip, s);
        else if (d0) nb = cheb_step<1, 1, kChebFused, DOT>(lv, f, dcur, dnext, x, out, j, partials, skip, s);
        else nb = cheb_step<1, 0, kChebFused, DOT>(lv, f, dcur, dnext, x, out, j, partials, skip, s);
        if (DOT) cheb_nparts_ = nb;
        return xi;
      }
      if (mode == kChebLast) {
        if (!zero) cheb_step<0, 0, kChebLast, 0>(lv, f, dcur, dnext, x, x, j, nullptr, skip, s);
        else if (d0) cheb_step<1, 1, kChebLast, 0>(lv, f, dcur, dnext, x, x, j, nullptr, skip, s);
        else cheb_step<1, 0, kChebLast, 0>(lv, f, dcur, dnext, x, x, j, nullptr, skip, s);
      } else {
        if (!zero) cheb_step<0, 0, kChebMid, 0>(lv, f, dcur, dnext, x, x, j, nullptr, skip, s);
        else if (d0) cheb_step<1, 1, kChebMid, 0>(lv, f, dcur, dnext, x, x, j, nullptr, skip, s);
        else cheb_step<1, 0, kChebMid, 0>(lv, f, dcur, dnext, x, x, j, nullptr, skip, s);
      }
      cur = zero ? 0 : 1 - cur;
    }
    return xi;
  }

  // The fused tail applies to one pre- and one post-sweep of a diagonal
  // smoother (the steps it reproduces); tail_first >= 1 was set at setup.
  bool use_tail() const {
    return h_->tail_first >= 1 && h_->tail_first < static_cast<int>(h_->lev.size()) && o_.npre == 1 &&
           o_.npost == 1 && o_.relax != AMG_CHEBYSHEV;
  }

  void launch_tail(int first, const int* skip, hipStream_t s) {
    const int nl = static_cast<int>(h_->lev.size());
    TailPlan<T> P{};
    P.nlev = nl - first;
    auto mat = [](const DevCsr<T>& M) { return TailMat<T>{M.view(), M.kind, M.lanes, M.bclass}; };
    for (int i = 0; i < P.nlev; ++i) {
      DevLevel<T>& lv = h_->lev[first + i];
      DevLevel<T>* next = (first + i + 1 < nl) ? &h_->lev[first + i + 1] : nullptr;
      TailLevel<T>& t = P.lev[i];
      t.A = mat(lv.A);
      t.P = mat(lv.P);
      t.R = mat(lv.R);
      t.f = lv.f;
      t.mf = lv.mf;
      t.m = lv.m;
      t.r = lv.r;
      t.y = lv.y;
      t.z = lv.z;
      t.fnext = next ? next->f : h_->fL;
      t.mfnext = next ? next->mf : nullptr;
      t.mnext = next ? next->m : nullptr;
    }
    P.Ainv = Ainv_;
    P.nL = nL_;
    P.fL = h_->fL;
    P.zL = h_->zL;
    P.sync = h_->tail_sync;
    P.limit = h_->tail_limit;
    vcycle_tail_kernel<T><<<h_->tail_grid, kBS, 0, s>>>(P, skip);
    AMG_LAUNCHED();
  }

  DevHierarchy<T>* h_;
  const double* Ainv_;
  int32_t nL_;
  VcycleOpts o_;
  int pre_cur_ = 0;
  int cheb_nparts_ = 0;
};

}  // namespace amg
