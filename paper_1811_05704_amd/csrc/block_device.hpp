// Block-value hierarchy on the device and its V-cycle (section 2, "AMG
// solve", with the 4 x 4 value type of section 3).
//
// Per level l < L (zero initial guess; with one pre- and one post-sweep of the
// block smoother M; post-sweeps apply M^T, the adjoint of the pre-sweep):
//   r_l     = f_l - A_l (M_l f_l)     level 1: (A_1 M_1) f_1 with the block
//                                      products A_ij M_j formed once at setup
//   f_{l+1} = R_l r_l                 restriction, with M_{l+1} f_{l+1}
//   ... z_L = A_L^-1 f_L (dense inverse of the scalar coarse matrix, FP64) ...
//   y_l     = M_l f_l + P_l z_{l+1}    prolongation + correction
//   z_l     = y_l + M_l^T (f_l - A_l y_l)   post-sweep (level 1 of PCG: r . z)
// Other sweep counts (0 .. 16 each) take an unfused form: the pre-sweeps
// z <- z + M (f - A z) from z = M f stored in a ping-pong pair, the residual
// of the last, and as many post-sweeps, the last writing the level's output.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <vector>

#include "block.hpp"
#include "block_setup.hpp"
#include "device.hpp"

namespace amg {

// Block rows above this mean length take 4 lanes per component.
constexpr double kBsrLongRow = 12.0;

template <class T>
struct DevBsr {
  int32_t rows = 0, cols = 0;  // block rows / columns
  int64_t nnzb = 0;
  int32_t* ptr = nullptr;
  int32_t* col = nullptr;
  T* val = nullptr;
  int sub = 1;  // lanes per block-row component
  BsrView<T> view() const { return BsrView<T>{ptr, col, val, rows}; }
  int blocks() const {
    const int rpb = kBS / (kB * sub);
    return (rows + rpb - 1) / rpb;
  }
};

template <class T>
hvec<T> bsr_values(const Bsr& M) {
  hvec<T> v(M.val.size());
  for_row_ranges(static_cast<int64_t>(v.size()), [&](int64_t b, int64_t e) {
    for (int64_t k = b; k < e; ++k) v[k] = static_cast<T>(M.val[k]);  // FP32: round to nearest
  });
  return v;
}

template <class T>
DevBsr<T> upload_bsr(DevArena& ar, const Bsr& M, const DevBsr<double>* like = nullptr) {
  DevBsr<T> d;
  d.rows = static_cast<int32_t>(M.rows);
  d.cols = static_cast<int32_t>(M.cols);
  d.nnzb = M.nnzb();
  if (like) {
    d.ptr = like->ptr;
    d.col = like->col;
  } else {
    std::vector<int32_t> p32(M.ptr.begin(), M.ptr.end());
    if (p32.empty()) p32.assign(1, 0);
    d.ptr = ar.upload(p32.data(), p32.size());
    d.col = ar.upload(M.col.data(), std::max<size_t>(M.col.size(), 1));
  }
  if constexpr (std::is_same<T, double>::value) {
    d.val = ar.upload(M.val.data(), std::max<size_t>(M.val.size(), 1));
  } else {
    const hvec<T> v = bsr_values<T>(M);
    d.val = ar.upload(v.data(), std::max<size_t>(v.size(), 1));
  }
  const double mean = M.rows ? double(M.nnzb()) / double(M.rows) : 0.0;
  d.sub = mean > kBsrLongRow ? 4 : 1;
  return d;
}

template <class T, class G, class E>
int launch_bsr(const DevBsr<T>& M, G g, E e, double* partials, const int* skip, hipStream_t s) {
  if (M.rows == 0) return 0;
  const int n = M.blocks();
  if (M.sub == 1) bsr_kernel<1, T, G, E><<<n, kBS, 0, s>>>(M.view(), g, e, partials, skip);
  else bsr_kernel<4, T, G, E><<<n, kBS, 0, s>>>(M.view(), g, e, partials, skip);
  AMG_LAUNCHED();
  return n;
}

template <class T>
struct DevBlockLevel {
  int32_t nb = 0;             // block rows (nodes)
  DevBsr<T> A, P, R;
  DevBsr<T> As;               // level 1: blocks A_ij M_j (same pattern as A)
  T* M = nullptr;             // smoother blocks, 16 per node
  T* f = nullptr;             // levels > 1: right-hand side
  T* mf = nullptr;            // levels > 1: M f, written by the restriction
  T* r = nullptr;
  T* y = nullptr;
  T* z = nullptr;             // levels > 1: output
  T* zp[2] = {nullptr, nullptr};  // pre-sweep iterates (sweep counts other than 1 / 1)
  T* t = nullptr;                 // post-sweep ping-pong partner (npost > 1)
};

// Level 1 first pre-sweep from zero, z = M f, one thread per scalar row
// (4 x 4 row times 4-vector in column order, as the restriction's M f).
template <class T, class TF>
static __global__ void __launch_bounds__(kVecBS) bscale_kernel(int n, T* z, const T* M, const TF* f,
                                                               const int* skip) {
  if (skip && *skip) return;
  const int stride = gridDim.x * kVecBS;
  for (int k = blockIdx.x * kVecBS + threadIdx.x; k < n; k += stride) {
    const int i = k / kB, q = k % kB;
    const T* m = M + static_cast<int64_t>(i) * kB2 + q * kB;
    const TF* fi = f + kB * i;
    T v = m[0] * static_cast<T>(fi[0]);
    v = v + m[1] * static_cast<T>(fi[1]);
    v = v + m[2] * static_cast<T>(fi[2]);
    v = v + m[3] * static_cast<T>(fi[3]);
    z[k] = v;
  }
}

// One more pre-sweep: out = z + M (f - A z), the row of M_i in column order.
template <class T, class TF>
struct EpiBPre {
  static constexpr int K = 0;
  T* out;
  const T* z;
  const T* M;
  const TF* f;
  __device__ __forceinline__ void operator()(int i, int q, const T* s4, double*) const {
    const T* m = M + static_cast<int64_t>(i) * kB2 + q * kB;
    const TF* fi = f + kB * i;
    T v = m[0] * (static_cast<T>(fi[0]) - s4[0]);
    v = v + m[1] * (static_cast<T>(fi[1]) - s4[1]);
    v = v + m[2] * (static_cast<T>(fi[2]) - s4[2]);
    v = v + m[3] * (static_cast<T>(fi[3]) - s4[3]);
    out[kB * i + q] = z[kB * i + q] + v;
  }
};

template <class T>
struct DevBlockHierarchy {
  std::vector<DevBlockLevel<T>> lev;  // levels 0 .. L-2
  T* fL = nullptr;                    // coarsest right-hand side / solution (scalar, 4 nb_L)
  T* zL = nullptr;
};

template <class T>
class BlockVcycle {
 public:
  BlockVcycle(DevBlockHierarchy<T>* h, const double* Ainv, int32_t nL, int npre = 1, int npost = 1)
      : h_(h), Ainv_(Ainv), nL_(nL), npre_(npre), npost_(npost) {}

  // z0 = V(f0); f0, z0 double[4 nb].  With DOT, writes the partials of
  // f0 . z0 and returns their count.
  template <int DOT>
  int run(const double* f0, double* z0, double* partials, const int* skip, hipStream_t s) {
    const int L = static_cast<int>(h_->lev.size()) + 1;
    if (L == 1) {
      coarse_gemv_kernel<double, double><<<nL_, kBS, 0, s>>>(nL_, Ainv_, f0, z0, skip);
      AMG_LAUNCHED();
      if (DOT) {
        const int nb = vec_blocks(nL_);
        dot_kernel<<<nb, kVecBS, 0, s>>>(nL_, f0, z0, partials, skip);
        AMG_LAUNCHED();
        return nb;
      }
      return 0;
    }
    if (npre_ != 1 || npost_ != 1) return run_sweeps<DOT>(f0, z0, partials, skip, s);
    for (int l = 0; l < L - 1; ++l) {
      DevBlockLevel<T>& lv = h_->lev[l];
      DevBlockLevel<T>* next = (l + 1 < L - 1) ? &h_->lev[l + 1] : nullptr;
      if (l == 0) {
        launch_bsr(lv.As, GatherX<T, double>{f0}, PerRow<EpiResid<T, double>>{{lv.r, f0}}, nullptr, skip, s);
      } else {
        launch_bsr(lv.A, GatherX<T, T>{lv.mf}, PerRow<EpiResid<T, T>>{{lv.r, lv.f}}, nullptr, skip, s);
      }
      if (next)
        launch_bsr(lv.R, GatherX<T, T>{lv.r}, EpiBRestrict<T>{next->f, next->mf, next->M}, nullptr, skip, s);
      else
        launch_bsr(lv.R, GatherX<T, T>{lv.r}, PerRow<EpiStore<T, T>>{{h_->fL}}, nullptr, skip, s);
    }
    coarse_gemv_kernel<T, T><<<nL_, kBS, 0, s>>>(nL_, Ainv_, h_->fL, h_->zL, skip);
    AMG_LAUNCHED();
    int nparts = 0;
    for (int l = L - 2; l >= 0; --l) {
      DevBlockLevel<T>& lv = h_->lev[l];
      const T* zc = (l + 1 < L - 1) ? h_->lev[l + 1].z : h_->zL;
      if (l == 0) {
        launch_bsr(lv.P, GatherX<T, T>{zc}, EpiBProlongMF<T, double>{lv.y, lv.M, f0}, nullptr, skip, s);
        nparts = launch_bsr(lv.A, GatherX<T, T>{lv.y}, EpiBSmooth<T, double, double, DOT>{z0, lv.y, lv.M, f0},
                            partials, skip, s);
      } else {
        launch_bsr(lv.P, GatherX<T, T>{zc}, PerRow<EpiProlong<T, T, 2>>{{lv.y, nullptr, nullptr, lv.mf}},
                   nullptr, skip, s);
        launch_bsr(lv.A, GatherX<T, T>{lv.y}, EpiBSmooth<T, T, T, 0>{lv.z, lv.y, lv.M, lv.f}, nullptr, skip, s);
      }
    }
    return DOT ? nparts : 0;
  }

 private:
  // The buffer holding level l's last pre-sweep (null with no pre-sweep):
  // the first is M f (level 1: bscale_kernel; deeper levels: written by the
  // restriction into mf), then each further sweep goes to the other of zp.
  T* pre_result(const DevBlockLevel<T>& lv, int l) const {
    if (npre_ == 0) return nullptr;
    T* cur = (l == 0) ? lv.zp[0] : lv.mf;
    for (int k = 1; k < npre_; ++k) cur = (cur == lv.zp[0]) ? lv.zp[1] : lv.zp[0];
    return cur;
  }

  template <class TF>
  void down_sweeps(DevBlockLevel<T>& lv, int l, const TF* f, DevBlockLevel<T>* next, const int* skip,
                   hipStream_t s) {
    auto restrict_from = [&](auto gather) {
      if (next && npre_ > 0)
        launch_bsr(lv.R, gather, EpiBRestrict<T>{next->f, next->mf, next->M}, nullptr, skip, s);
      else
        launch_bsr(lv.R, gather, PerRow<EpiStore<T, T>>{{next ? next->f : h_->fL}}, nullptr, skip, s);
    };
    if (npre_ == 0) {
      restrict_from(GatherX<T, TF>{f});
      return;
    }
    T* cur = lv.mf;
    if (l == 0) {
      const int n = kB * lv.nb;
      bscale_kernel<T, TF><<<vec_blocks(n), kVecBS, 0, s>>>(n, lv.zp[0], lv.M, f, skip);
      AMG_LAUNCHED();
      cur = lv.zp[0];
    }
    for (int k = 1; k < npre_; ++k) {
      T* dst = (cur == lv.zp[0]) ? lv.zp[1] : lv.zp[0];
      launch_bsr(lv.A, GatherX<T, T>{cur}, EpiBPre<T, TF>{dst, cur, lv.M, f}, nullptr, skip, s);
      cur = dst;
    }
    launch_bsr(lv.A, GatherX<T, T>{cur}, PerRow<EpiResid<T, TF>>{{lv.r, f}}, nullptr, skip, s);
    restrict_from(GatherX<T, T>{lv.r});
  }

  template <class TF, class TZ, int DOT>
  int up_sweeps(DevBlockLevel<T>& lv, int l, const TF* f, const T* zc, TZ* zout, double* partials,
                const int* skip, hipStream_t s) {
    if (npre_ == 0)
      launch_bsr(lv.P, GatherX<T, T>{zc}, PerRow<EpiProlong<T, T, 0>>{{lv.y, nullptr, nullptr, nullptr}}, nullptr,
                 skip, s);
    else
      launch_bsr(lv.P, GatherX<T, T>{zc}, PerRow<EpiProlong<T, T, 2>>{{lv.y, nullptr, nullptr, pre_result(lv, l)}},
                 nullptr, skip, s);
    if (npost_ == 0) {
      const int n = kB * lv.nb, nb = vec_blocks(n);
      copy_dot_kernel<T, TF, TZ, DOT><<<nb, kVecBS, 0, s>>>(n, zout, lv.y, f, partials, skip);
      AMG_LAUNCHED();
      return DOT ? nb : 0;
    }
    T* cur = lv.y;
    T* other = lv.t;
    int nparts = 0;
    for (int k = 0; k < npost_; ++k) {
      if (k == npost_ - 1) {
        nparts = launch_bsr(lv.A, GatherX<T, T>{cur}, EpiBSmooth<T, TF, TZ, DOT>{zout, cur, lv.M, f}, partials,
                            skip, s);
      } else {
        launch_bsr(lv.A, GatherX<T, T>{cur}, EpiBSmooth<T, TF, T, 0>{other, cur, lv.M, f}, nullptr, skip, s);
        std::swap(cur, other);
      }
    }
    return DOT ? nparts : 0;
  }

  template <int DOT>
  int run_sweeps(const double* f0, double* z0, double* partials, const int* skip, hipStream_t s) {
    const int L = static_cast<int>(h_->lev.size()) + 1;
    for (int l = 0; l < L - 1; ++l) {
      DevBlockLevel<T>& lv = h_->lev[l];
      DevBlockLevel<T>* next = (l + 1 < L - 1) ? &h_->lev[l + 1] : nullptr;
      if (l == 0) down_sweeps<double>(lv, l, f0, next, skip, s);
      else down_sweeps<T>(lv, l, lv.f, next, skip, s);
    }
    coarse_gemv_kernel<T, T><<<nL_, kBS, 0, s>>>(nL_, Ainv_, h_->fL, h_->zL, skip);
    AMG_LAUNCHED();
    int nparts = 0;
    for (int l = L - 2; l >= 0; --l) {
      DevBlockLevel<T>& lv = h_->lev[l];
      const T* zc = (l + 1 < L - 1) ? h_->lev[l + 1].z : h_->zL;
      if (l == 0) nparts = up_sweeps<double, double, DOT>(lv, l, f0, zc, z0, partials, skip, s);
      else up_sweeps<T, T, 0>(lv, l, lv.f, zc, lv.z, partials, skip, s);
    }
    return DOT ? nparts : 0;
  }

  DevBlockHierarchy<T>* h_;
  const double* Ainv_;
  int32_t nL_;
  int npre_, npost_;
};

// Level matrices, smoother blocks and vectors of a block hierarchy.  The
// FP64 fine operator B0 (the Krylov loop's) shares its pattern with level 1.
template <class T>
inline void upload_block_levels(DevArena& ar, const BlockHierarchy& H, const DevBsr<double>& B0,
                                DevBlockHierarchy<T>& D, int npre = 1, int npost = 1) {
  const int L = static_cast<int>(H.levels.size());
  for (int l = 0; l < L - 1; ++l) {
    const BlockLevel& hl = H.levels[l];
    DevBlockLevel<T> d;
    d.nb = static_cast<int32_t>(hl.A.rows);
    if constexpr (std::is_same<T, double>::value) d.A = (l == 0) ? B0 : upload_bsr<T>(ar, hl.A);
    else d.A = upload_bsr<T>(ar, hl.A, l == 0 ? &B0 : nullptr);
    d.P = upload_bsr<T>(ar, hl.P);
    d.R = upload_bsr<T>(ar, hl.R);
    std::vector<T> m(hl.M.begin(), hl.M.end());
    d.M = ar.upload(m.data(), m.size());
    if (l == 0) {
      // (A M)_ij = A_ij M_j, block products in c order, FP64 then rounded;
      // the pattern is B0's, so only the values are formed
      Bsr AM;
      AM.rows = hl.A.rows;
      AM.cols = hl.A.cols;
      AM.ptr = hl.A.ptr;
      AM.val.resize(hl.A.val.size());
      for_row_ranges(hl.A.rows, [&](int64_t b, int64_t end) {
        for (int64_t i = b; i < end; ++i)
          for (int64_t e = hl.A.ptr[i]; e < hl.A.ptr[i + 1]; ++e) {
            const double* a = &hl.A.val[e * kB2];
            const double* mj = &hl.M[static_cast<int64_t>(hl.A.col[e]) * kB2];
            double* o = &AM.val[e * kB2];
            for (int r = 0; r < kB; ++r)
              for (int c = 0; c < kB; ++c) {
                double t = a[r * kB] * mj[c];
                for (int k = 1; k < kB; ++k) t = t + a[r * kB + k] * mj[k * kB + c];
                o[r * kB + c] = t;
              }
          }
      });
      d.As = upload_bsr<T>(ar, AM, &B0);
    }
    AMG_HIP(hipStreamSynchronize(ar.stream()));
    const int64_t n = int64_t(kB) * d.nb;
    if (l > 0) {
      d.f = ar.get<T>(n);
      d.mf = ar.get<T>(n);
      d.z = ar.get<T>(n);
    }
    d.r = ar.get<T>(n);
    d.y = ar.get<T>(n);
    if ((npre != 1 || npost != 1) && npre > 0) {
      d.zp[0] = ar.get<T>(n);
      d.zp[1] = ar.get<T>(n);
    }
    if (npost > 1) d.t = ar.get<T>(n);
    D.lev.push_back(d);
  }
  const int64_t nL = int64_t(kB) * H.levels.back().A.rows;
  if (L > 1) {
    D.fL = ar.get<T>(nL);
    D.zL = ar.get<T>(nL);
  }
}

}  // namespace amg
