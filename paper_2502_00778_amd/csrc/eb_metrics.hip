// Lumped directed-area vectors, boundary dual normals and dual volumes.
//
//   n_jk = 2/(D(D+1)) sum_{E contains jk} n_j^E  (j = tail = smaller id)
//          + 1/(D(D+1)) sum_{B contains jk} n_B  (eq.
//          efficient_njk_formula_general_D and the boundary correction)
//   b_j  = (1/D) sum_{B contains j} n_B          (closure, Section 3.2.3)
//   V_j  = sum_{E contains j} |E|/(D+1)          (Section 4.2)
//   V_j  = 1/(2D) sum_k (x_k - x_j).n_jk         (edge loop, Section 4.1)
//
// Two reductions:
//   atomic  one thread per element (and per boundary face); FP64 atomic adds
//           into zeroed n, V, b.
//   gather  one thread per node j.  It walks j's elements in node_inc order,
//           forms the one face vector n_j^E each element needs for the edges
//           whose tail is j (the paper's remark that n_j^E serves every edge
//           leaving j, Section 3.3), and |E| from the same cross product; the
//           edges with tail j are a contiguous range owned by j's block, which
//           accumulates them in LDS and writes them once, coalesced.  No
//           memset, no atomics, a fixed summation order: bitwise reproducible.
#include "eb_gather.h"

namespace eb {

// ------------------------------------------------------------- atomic path

// One thread per element: the outward face normals and |E|, then
// n_e += 2/(D(D+1)) n_tail^E for each local edge and V_i += |E|/(D+1) for
// each vertex, summed per edge and node in the block's LDS tables and added
// to the zeroed outputs with one FP64 atomic per distinct edge or node and
// component.  n and vol may be null (skipped).
template <int D>
__global__ __launch_bounds__(ATOMIC_TB) void k_fwd_atomic_elem(FwdArgs a) {
  constexpr int NN = D + 1, NE = EL<D>::NE;
  __shared__ LdsAcc<ATOMIC_HE, D> te;
  __shared__ LdsAcc<ATOMIC_HV, 1> tv;
  const int t = threadIdx.x;
  const bool want_n = a.n_x != nullptr, want_v = a.vol != nullptr;
  double *const nout[3] = {a.n_x, a.n_y, a.n_z};
  double *const vout[1] = {a.vol};
  if (want_n) lds_acc_init<ATOMIC_TB>(te, t);
  if (want_v) lds_acc_init<ATOMIC_TB>(tv, t);
  __syncthreads();
  const int64_t e0 = (int64_t)blockIdx.x * ATOMIC_TB * ATOMIC_EPT;
#pragma unroll
  for (int k = 0; k < ATOMIC_EPT; ++k) {
    const int64_t e = e0 + (int64_t)k * ATOMIC_TB + t;
    if (e >= a.nelem) break;
    int32_t v[NN];
    load_conn<D>(a.elem, e, v);
    V3 P[NN], n[NN];
#pragma unroll
    for (int i = 0; i < NN; ++i) P[i] = load_pt<D>(a.X, v[i]);
    const double det = elem_normals<D>(P, n);
    if (det == 0.0) raise_status(a.st, EB_EDEGENERATE, e);
    constexpr double kN = 2.0 / (D * (D + 1));
    if (want_n) {
#pragma unroll
      for (int le = 0; le < NE; ++le) {
        const int p = pair_p<D>(le), q = pair_q<D>(le);
        const V3 nt = v[p] < v[q] ? n[p] : n[q];
        double c[D];
        c[0] = kN * nt.x;
        c[1] = kN * nt.y;
        if constexpr (D == 3) c[D - 1] = kN * nt.z;
        lds_acc_add(te, nout, a.elem_edge[e * NE + le], c);
      }
    }
    if (want_v) {
      const double share[1] = {D == 3 ? fabs(det) / 24.0 : fabs(det) / 6.0};
#pragma unroll
      for (int i = 0; i < NN; ++i) lds_acc_add(tv, vout, v[i], share);
    }
  }
  __syncthreads();
  if (want_n) lds_acc_flush<ATOMIC_TB>(te, nout, t);
  if (want_v) lds_acc_flush<ATOMIC_TB>(tv, vout, t);
}

// One thread per boundary face; a block's faces (in bface order, consecutive
// ones sharing most vertices and edges) sum n_B/(D(D+1)) per edge and n_B/D
// per boundary node in LDS tables first, then add each sum with one FP64
// atomic per component.
constexpr int AB_TB = 256, AB_HE = 1024, AB_HB = 512;

template <int D>
__global__ __launch_bounds__(AB_TB) void k_fwd_atomic_bface(FwdArgs a) {
  __shared__ LdsAcc<AB_HE, D> te;
  __shared__ LdsAcc<AB_HB, D> tb;
  const int t = threadIdx.x;
  const bool want_n = a.n_x != nullptr, want_b = a.b_x != nullptr;
  double *const nout[3] = {a.n_x, a.n_y, a.n_z};
  double *const bout[3] = {a.b_x, a.b_y, a.b_z};
  if (want_n) lds_acc_init<AB_TB>(te, t);
  if (want_b) lds_acc_init<AB_TB>(tb, t);
  __syncthreads();
  const int64_t f = (int64_t)blockIdx.x * AB_TB + t;
  if (f < a.nbface) {
    V3 nB;
    int32_t fv[D];
#pragma unroll
    for (int s = 0; s < D; ++s) fv[s] = a.bface[f * D + s];
    if constexpr (D == 3) {
      const V3 A = load_pt<D>(a.X, fv[0]), B = load_pt<D>(a.X, fv[1]), C = load_pt<D>(a.X, fv[2]);
      nB = 0.5 * cross(B - A, C - A);
    } else {
      nB = rot2(load_pt<D>(a.X, fv[1]) - load_pt<D>(a.X, fv[0]));
    }
    constexpr int NBE = D == 2 ? 1 : 3;
    if (want_n) {
      constexpr double kB = 1.0 / (D * (D + 1));
      double c[D];
      c[0] = kB * nB.x;
      c[1] = kB * nB.y;
      if constexpr (D == 3) c[D - 1] = kB * nB.z;
#pragma unroll
      for (int i = 0; i < NBE; ++i) lds_acc_add(te, nout, a.bface_edge[f * NBE + i], c);
    }
    if (want_b) {
      constexpr double kb = 1.0 / D;
      double c[D];
      c[0] = kb * nB.x;
      c[1] = kb * nB.y;
      if constexpr (D == 3) c[D - 1] = kb * nB.z;
#pragma unroll
      for (int s = 0; s < D; ++s) lds_acc_add(tb, bout, a.node_bnode[fv[s]], c);
    }
  }
  __syncthreads();
  if (want_n) lds_acc_flush<AB_TB>(te, nout, t);
  if (want_b) lds_acc_flush<AB_TB>(tb, bout, t);
}

// ------------------------------------------------------------- gather path
// (device bodies in eb_gather.h)

template <int D, int TN, int CAP, int U, bool WIDE, int VAR>
__global__ __launch_bounds__(TN) void k_fwd_gather_variant(FwdArgs a) {
  __shared__ double acc[D][CAP];
  fwd_node_tile<D, TN, CAP, U, WIDE, VAR>(a, tile_of_block(gridDim.x, a.xcd_remap), acc);
}

// Traditional boundary loop: b_j from node j's share of each boundary face
// built from the edge midpoints and the face centroid (Section 3.2), each
// piece oriented like the face's outward normal.  The dual-face pieces of
// the interior loop already sum to the corrected n, so n is left alone.
template <int D>
__global__ __launch_bounds__(256) void k_fwd_boundary_dual(FwdArgs a) {
  const int64_t bj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (bj >= a.nbnode || !a.b_x) return;
  const int32_t j = a.bnode[bj];
  V3 bs = {0.0, 0.0, 0.0};
  for (int32_t r = a.bnode_face_off[bj]; r < a.bnode_face_off[bj + 1]; ++r) {
    const int32_t f = a.bnode_face[r];
    int32_t fv[D];
#pragma unroll
    for (int s = 0; s < D; ++s) fv[s] = a.bface[(int64_t)f * D + s];
    if constexpr (D == 3) {
      const V3 A = load_pt<D>(a.X, fv[0]), B = load_pt<D>(a.X, fv[1]), C = load_pt<D>(a.X, fv[2]);
      const V3 nB = cross(B - A, C - A);
      const V3 xi = fv[0] == j ? A : (fv[1] == j ? B : C);
      const V3 xa = fv[0] == j ? B : A, xb = fv[2] == j ? B : C;
      const V3 G = (1.0 / 3.0) * (A + B + C), ma = 0.5 * (xi + xa), mb = 0.5 * (xi + xb);
      V3 t1 = 0.5 * cross(ma - xi, G - xi), t2 = 0.5 * cross(G - xi, mb - xi);
      if (dot(t1, nB) < 0.0) t1 = -t1;
      if (dot(t2, nB) < 0.0) t2 = -t2;
      bs = bs + t1 + t2;
    } else {
      const V3 A = load_pt<D>(a.X, fv[0]), B = load_pt<D>(a.X, fv[1]);
      const V3 nB = rot2(B - A);
      const V3 xi = fv[0] == j ? A : B, xo = fv[0] == j ? B : A;
      V3 t = rot2(0.5 * (xi + xo) - xi);
      if (dot(t, nB) < 0.0) t = -t;
      bs = bs + t;
    }
  }
  a.b_x[bj] = bs.x;
  a.b_y[bj] = bs.y;
  if (D == 3) a.b_z[bj] = bs.z;
}

// The boundary pass with BG lanes per boundary node: the node's faces are
// formed a lane each, BG_FACES at a time staged in LDS; then a lane per
// out-edge adds n_B/(D(D+1)) of the faces holding the edge's head, in face
// order, and the group's first lane sums b_j's n_B in face order: per output
// the operations, in the order, of fwd_boundary_node (the persistent
// kernel's form; both uncontracted, so their bits agree).
constexpr int BG = 8, BG_FACES = 16;

template <int D>
__global__ __launch_bounds__(64) void k_fwd_boundary_gather(FwdArgs a) {
  __shared__ int32_t sfv[64 / BG][BG_FACES][D];
  __shared__ double snb[64 / BG][BG_FACES][3];
  const int t = threadIdx.x, grp = t / BG, g = t % BG;
  const int64_t bj = (int64_t)blockIdx.x * (64 / BG) + grp;
  const bool live = bj < a.nbnode;
  int32_t j = 0, my0 = 0, nout = 0, r0 = 0, nf = 0;
  if (live) {
    j = a.bnode[bj];
    my0 = a.node_edge_off[j];
    nout = a.node_edge_off[j + 1] - my0;
    r0 = a.bnode_face_off[bj];
    nf = a.bnode_face_off[bj + 1] - r0;
  }
  // chunks of faces, as many as the block's longest list needs (every lane
  // takes every barrier)
  int32_t nch = (nf + BG_FACES - 1) / BG_FACES;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) nch = max(nch, __shfl_xor(nch, o, 64));
  constexpr double kB = 1.0 / (D * (D + 1));
  V3 bs = {0.0, 0.0, 0.0};
  for (int32_t ch = 0; ch < nch; ++ch) {
    const int32_t u0 = ch * BG_FACES, m = min(nf - u0, BG_FACES);
    __syncthreads();  // (the previous chunk is used up)
    for (int32_t u = g; u < m; u += BG) {
      const int32_t f = a.bnode_face[r0 + u0 + u];
      V3 P[D];
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const int32_t v = a.bface[(int64_t)f * D + q];
        sfv[grp][u][q] = v;
        P[q] = load_pt<D>(a.X, v);
      }
      V3 nB;
      if constexpr (D == 3)
        nB = nc_scale(0.5, nc_cross(P[1] - P[0], P[2] - P[0]));
      else
        nB = rot2(P[1] - P[0]);
      snb[grp][u][0] = nB.x;
      snb[grp][u][1] = nB.y;
      snb[grp][u][2] = nB.z;
    }
    __syncthreads();
    if (g == 0)
      for (int32_t u = 0; u < m; ++u)
        bs = nc_add(bs, V3{snb[grp][u][0], snb[grp][u][1], snb[grp][u][2]});
    for (int32_t q = g; q < nout; q += BG) {
      const int32_t e = my0 + q, h = a.edge_head[e];
      V3 acc = {0.0, 0.0, 0.0};
      bool any = false;
      for (int32_t u = 0; u < m; ++u) {
        bool on = false;
#pragma unroll
        for (int k = 0; k < D; ++k) on = on || sfv[grp][u][k] == h;
        if (!on) continue;
        if (!any) {
          acc = V3{a.n_x[e], a.n_y[e], D == 3 ? a.n_z[e] : 0.0};
          any = true;
        }
        acc = nc_add(acc, nc_scale(kB, V3{snb[grp][u][0], snb[grp][u][1], snb[grp][u][2]}));
      }
      if (any) {
        a.n_x[e] = acc.x;
        a.n_y[e] = acc.y;
        if (D == 3) a.n_z[e] = acc.z;
      }
    }
  }
  if (live && g == 0 && a.b_x) {
    const V3 bo = nc_scale(1.0 / D, bs);
    a.b_x[bj] = bo.x;
    a.b_y[bj] = bo.y;
    if (D == 3) a.b_z[bj] = bo.z;
  }
}

// ----------------------------------------------------- volumes on their own

template <int D>
__global__ __launch_bounds__(256) void k_vol_elem_gather(FwdArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.nv) return;
  double vs = 0.0;
  for (int32_t r = a.node_inc_off[j]; r < a.node_inc_off[j + 1]; ++r) {
    const int64_t e = a.node_inc[r] / (D + 1);
    int32_t v[D + 1];
    load_conn<D>(a.elem, e, v);
    V3 P[D + 1], n[D + 1];
#pragma unroll
    for (int i = 0; i <= D; ++i) P[i] = load_pt<D>(a.X, v[i]);
    vs += fabs(elem_normals<D>(P, n));
  }
  a.vol[j] = vs * (D == 3 ? 1.0 / 24.0 : 1.0 / 6.0);
}

template <int D>
__global__ __launch_bounds__(256) void k_vol_edge_atomic(FwdArgs a, const double *__restrict__ nx,
                                                         const double *__restrict__ ny,
                                                         const double *__restrict__ nz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nedge) return;
  const int32_t j = a.edge_tail[e], k = a.edge_head[e];
  const V3 d = load_pt<D>(a.X, k) - load_pt<D>(a.X, j);
  double s = d.x * nx[e] + d.y * ny[e];
  if (D == 3) s += d.z * nz[e];
  s *= 1.0 / (2 * D);
  unsafeAtomicAdd(&a.vol[j], s);
  unsafeAtomicAdd(&a.vol[k], s);
}

// Edge loop in two passes: each edge's term t_e = (x_k - x_j).n_jk / (2D)
// once (coalesced over edges), then each node sums the terms of its out-edges
// (a contiguous range) and in-edges (node_in order): fixed order, no atomics.
template <int D>
__global__ __launch_bounds__(256) void k_vol_edge_terms(FwdArgs a, const double *__restrict__ nx,
                                                        const double *__restrict__ ny,
                                                        const double *__restrict__ nz,
                                                        double *__restrict__ term) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nedge) return;
  const V3 d = load_pt<D>(a.X, a.edge_head[e]) - load_pt<D>(a.X, a.edge_tail[e]);
  term[e] = (d.x * nx[e] + d.y * ny[e] + (D == 3 ? d.z * nz[e] : 0.0)) * (1.0 / (2 * D));
}

__global__ __launch_bounds__(256) void k_vol_edge_sum(FwdArgs a, const double *__restrict__ term) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.nv) return;
  double s = sum_terms<false>(0.0, term, a.node_edge_off[j], a.node_edge_off[j + 1]);
  s = sum_terms_at<false>(s, term, a.node_in_edge, a.node_in_off[j], a.node_in_off[j + 1]);
  a.vol[j] = s;
}

// ------------------------------------------------- edge-loop residual
// The consumer of the metrics (the edge-based discretization of Section 2):
// Res_j = sum over edges (j,k) of phi_jk, with phi_jk = (F_j + F_k)/2 . n_jk
// added at the tail and subtracted at the head, plus the boundary flux of
// j's boundary faces.  Two passes like the edge loop: per-edge phi_e, then
// per node the ordered sum; then boundary nodes add their faces in order.

template <int D>
__global__ __launch_bounds__(256) void k_res_edge_terms(FwdArgs a, const double *__restrict__ nx,
                                                        const double *__restrict__ ny,
                                                        const double *__restrict__ nz,
                                                        const double *__restrict__ F,
                                                        double *__restrict__ term) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.nedge) return;
  const int32_t j = a.edge_tail[e], k = a.edge_head[e];
  const int64_t nv = a.nv;
  double s = (F[j] + F[k]) * nx[e] + (F[nv + j] + F[nv + k]) * ny[e];
  if (D == 3) s += (F[2 * nv + j] + F[2 * nv + k]) * nz[e];
  term[e] = 0.5 * s;
}

__global__ __launch_bounds__(256) void k_res_node_sum(FwdArgs a, const double *__restrict__ term,
                                                      double *__restrict__ res) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.nv) return;
  double s = sum_terms<false>(0.0, term, a.node_edge_off[j], a.node_edge_off[j + 1]);
  s = sum_terms_at<true>(s, term, a.node_in_edge, a.node_in_off[j], a.node_in_off[j + 1]);
  res[j] = s;
}

// Boundary flux of boundary node bj.  NODE: F_j . b_j.  LINEAR: per face B,
// n_B/D times F at the weights (2D: 5/6 own, 1/6 other; 3D: 6/8 own, 1/8 each
// other), which makes the residual exact for linear F at every node.
template <int D, bool LINEAR>
__global__ __launch_bounds__(256) void k_res_boundary(FwdArgs a, const double *__restrict__ F,
                                                      double *__restrict__ res) {
  const int64_t bj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (bj >= a.nbnode) return;
  const int32_t j = a.bnode[bj];
  const int64_t nv = a.nv;
  auto Fat = [&](int32_t i) {
    return V3{F[i], F[nv + i], D == 3 ? F[2 * nv + i] : 0.0};
  };
  double s = 0.0;
  if constexpr (!LINEAR) {
    const V3 b = {a.b_x[bj], a.b_y[bj], D == 3 ? a.b_z[bj] : 0.0};
    s = dot(Fat(j), b);
  } else {
    for (int32_t r = a.bnode_face_off[bj]; r < a.bnode_face_off[bj + 1]; ++r) {
      const int32_t f = a.bnode_face[r];
      int32_t fv[D];
#pragma unroll
      for (int q = 0; q < D; ++q) fv[q] = a.bface[(int64_t)f * D + q];
      V3 nB, Fq;
      if constexpr (D == 3) {
        const V3 A = load_pt<D>(a.X, fv[0]), B = load_pt<D>(a.X, fv[1]), C = load_pt<D>(a.X, fv[2]);
        nB = (1.0 / 6.0) * cross(B - A, C - A);  // n_B / D
        const V3 F0 = Fat(fv[0]), F1 = Fat(fv[1]), F2 = Fat(fv[2]);
        const V3 sum = F0 + F1 + F2, own = fv[0] == j ? F0 : (fv[1] == j ? F1 : F2);
        Fq = 0.125 * (sum + 5.0 * own);
      } else {
        nB = 0.5 * rot2(load_pt<D>(a.X, fv[1]) - load_pt<D>(a.X, fv[0]));  // n_B / D
        const V3 F0 = Fat(fv[0]), F1 = Fat(fv[1]);
        const V3 own = fv[0] == j ? F0 : F1, other = fv[0] == j ? F1 : F0;
        Fq = (1.0 / 6.0) * (5.0 * own + other);
      }
      s += dot(Fq, nB);
    }
  }
  res[j] += s;
}

template <int D>
int residual_impl(const FwdArgs &a, const double *n_edge, const double *F, int linear,
                  double *res, hipStream_t s) {
  const double *nx = n_edge, *ny = n_edge + a.nedge, *nz = D == 3 ? n_edge + 2 * a.nedge : nullptr;
  if (a.nedge > 0) {
    launch_principal(k_res_edge_terms<D>, dim3(grid_for(a.nedge, 256)), dim3(256), 0, s, a, nx,
                     ny, nz, F, a.vterm);
    EB_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_res_node_sum, dim3(grid_for(a.nv, 256)), dim3(256), 0, s, a,
                     (const double *)a.vterm, res);
  EB_LAUNCH_CHECK();
  if (a.nbnode > 0) {
    if (linear)
      hipLaunchKernelGGL((k_res_boundary<D, true>), dim3(grid_for(a.nbnode, 256)), dim3(256), 0,
                         s, a, F, res);
    else
      hipLaunchKernelGGL((k_res_boundary<D, false>), dim3(grid_for(a.nbnode, 256)), dim3(256), 0,
                         s, a, F, res);
    EB_LAUNCH_CHECK();
  }
  return EB_OK;
}

template int residual_impl<2>(const FwdArgs &, const double *, const double *, int, double *,
                              hipStream_t);
template int residual_impl<3>(const FwdArgs &, const double *, const double *, int, double *,
                              hipStream_t);

// ------------------------------------------------------------- launchers

template <int D> int launch_fwd_boundary(const FwdArgs &a, hipStream_t s);

template <int D>
int launch_fwd_gather(const FwdArgs &a, const LaunchCfg &cfg, hipStream_t s) {
  EB_TRY(launch_fwd_nodes<D>(a, cfg, s));
  return launch_fwd_boundary<D>(a, s);
}

template <int D>
int launch_fwd_boundary(const FwdArgs &a, hipStream_t s) {
  if (a.nbnode <= 0) return EB_OK;
  // (blocks of one wave: the few boundary nodes spread over every CU)
  launch_span(k_fwd_boundary_gather<D>, dim3(grid_for(a.nbnode, 64 / BG)), dim3(64), 0, s, a);
  EB_LAUNCH_CHECK();
  return EB_OK;
}

template <int D>
int forward_variant_impl(const FwdArgs &a, int variant, const LaunchCfg &cfg, hipStream_t s) {
  if (variant == 0) return launch_fwd_gather<D>(a, cfg, s);
  // one shape (128 nodes, chunks of 4, XCD order as set): for comparison
  const dim3 grid((unsigned)((a.nv + 127) / 128));
  if (a.sell_wide) {
    if (variant == 1)
      launch_principal((k_fwd_gather_variant<D, 128, 1024, 4, true, VAR_EDGE>), grid, dim3(128), 0,
                       s, a);
    else
      launch_principal((k_fwd_gather_variant<D, 128, 1024, 4, true, VAR_DUAL>), grid, dim3(128), 0,
                       s, a);
  } else {
    if (variant == 1)
      launch_principal((k_fwd_gather_variant<D, 128, 1024, 4, false, VAR_EDGE>), grid, dim3(128),
                       0, s, a);
    else
      launch_principal((k_fwd_gather_variant<D, 128, 1024, 4, false, VAR_DUAL>), grid, dim3(128),
                       0, s, a);
  }
  EB_LAUNCH_CHECK();
  if (a.nbnode <= 0) return EB_OK;
  if (variant == 1) return launch_fwd_boundary<D>(a, s);
  hipLaunchKernelGGL(k_fwd_boundary_dual<D>, dim3(grid_for(a.nbnode, 256)), dim3(256), 0, s, a);
  EB_LAUNCH_CHECK();
  return EB_OK;
}

template int forward_variant_impl<2>(const FwdArgs &, int, const LaunchCfg &, hipStream_t);
template int forward_variant_impl<3>(const FwdArgs &, int, const LaunchCfg &, hipStream_t);

template <int D>
int forward_impl(const FwdArgs &a, int reduce, const LaunchCfg &cfg, hipStream_t s) {
  if (reduce == EB_REDUCE_ATOMIC) {
    if (a.n_x) {
      EB_TRY(fill_f64(a.n_x, a.nedge, 0.0, s));
      EB_TRY(fill_f64(a.n_y, a.nedge, 0.0, s));
      if (D == 3) EB_TRY(fill_f64(a.n_z, a.nedge, 0.0, s));
    }
    if (a.vol) EB_TRY(fill_f64(a.vol, a.nv, 0.0, s));
    if (a.b_x) {
      EB_TRY(fill_f64(a.b_x, a.nbnode, 0.0, s));
      EB_TRY(fill_f64(a.b_y, a.nbnode, 0.0, s));
      if (D == 3) EB_TRY(fill_f64(a.b_z, a.nbnode, 0.0, s));
    }
    if (a.nelem > 0) {
      launch_principal(k_fwd_atomic_elem<D>, dim3(grid_for(a.nelem, ATOMIC_TB * ATOMIC_EPT)),
                       dim3(ATOMIC_TB), 0, s,
                         a);
      EB_LAUNCH_CHECK();
    }
    if (a.nbface > 0 && (a.n_x || a.b_x)) {
      launch_span(k_fwd_atomic_bface<D>, dim3(grid_for(a.nbface, AB_TB)), dim3(AB_TB), 0, s, a);
      EB_LAUNCH_CHECK();
    }
    return EB_OK;
  }
  return launch_fwd_gather<D>(a, cfg, s);
}

template int forward_impl<2>(const FwdArgs &, int, const LaunchCfg &, hipStream_t);
template int forward_impl<3>(const FwdArgs &, int, const LaunchCfg &, hipStream_t);

template <int D>
int volumes_impl(const FwdArgs &a, int mode, int reduce, const double *n_edge, hipStream_t s) {
  if (mode == EB_VOL_ELEMENT) {
    if (reduce == EB_REDUCE_ATOMIC) {
      FwdArgs b = a;
      b.n_x = b.n_y = b.n_z = nullptr;
      b.b_x = b.b_y = b.b_z = nullptr;
      EB_TRY(fill_f64(b.vol, b.nv, 0.0, s));
      if (b.nelem > 0) {
        launch_principal(k_fwd_atomic_elem<D>, dim3(grid_for(b.nelem, ATOMIC_TB * ATOMIC_EPT)),
                         dim3(ATOMIC_TB), 0, s, b);
        EB_LAUNCH_CHECK();
      }
      return EB_OK;
    }
    launch_principal(k_vol_elem_gather<D>, dim3(grid_for(a.nv, 256)), dim3(256), 0, s, a);
    EB_LAUNCH_CHECK();
    return EB_OK;
  }
  const double *nx = n_edge, *ny = n_edge + a.nedge, *nz = D == 3 ? n_edge + 2 * a.nedge : nullptr;
  if (reduce == EB_REDUCE_ATOMIC) {
    EB_TRY(fill_f64(a.vol, a.nv, 0.0, s));
    if (a.nedge > 0) {
      launch_principal(k_vol_edge_atomic<D>, dim3(grid_for(a.nedge, 256)), dim3(256), 0, s, a,
                         nx, ny, nz);
      EB_LAUNCH_CHECK();
    }
    return EB_OK;
  }
  if (!a.vterm) {
    set_detail("the gather edge loop needs the workspace's term buffer");
    return EB_EINVAL;
  }
  if (a.nedge > 0) {
    launch_principal(k_vol_edge_terms<D>, dim3(grid_for(a.nedge, 256)), dim3(256), 0, s, a, nx,
                     ny, nz, a.vterm);
    EB_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_vol_edge_sum, dim3(grid_for(a.nv, 256)), dim3(256), 0, s, a,
                     (const double *)a.vterm);
  EB_LAUNCH_CHECK();
  return EB_OK;
}

template int volumes_impl<2>(const FwdArgs &, int, int, const double *, hipStream_t);
template int volumes_impl<3>(const FwdArgs &, int, int, const double *, hipStream_t);

}  // namespace eb
