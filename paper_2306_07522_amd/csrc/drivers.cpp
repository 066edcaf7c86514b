// C ABI drivers: RK4 propagation (Fig. 1d, time evolution), stationary
// state (Fig. 1d, stationary states) and spectra (Methods, "Numerical
// computation of the spectrum").
#include <chrono>
#include <cmath>
#include <cstring>

#include "blas.h"
#include "internal.h"
#include "nn.h"
#include "solvers.h"

namespace heom {

static const double kPi = 3.14159265358979323846;

template <typename T>
static heom_status vec_norm(const void *v, int64_t n, int R, double2 *partial, int nchunk, double2 *hdev, PinnedBuf &pin,
                            std::vector<double> &out, hipStream_t s) {
  HEOM_TRY(mdot<T>(v, 0, 1, v, n, R, partial, nchunk, hdev, s));
  HEOM_TRY(pin.ensure(sizeof(double2) * R));
  HEOM_HIP_CHECK(hipMemcpyAsync(pin.p, hdev, sizeof(double2) * R, hipMemcpyDeviceToHost, s));
  HEOM_HIP_CHECK(hipStreamSynchronize(s));
  out.resize(R);
  for (int r = 0; r < R; ++r) out[r] = std::sqrt(std::max(((double2 *)pin.p)[r].x, 0.0));
  return HEOM_OK;
}

static int nchunk_for(int64_t n, int R) {
  int64_t c = (n * R) / (256 * 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(c, 1024));
}

// Linear system (M + diag(shifts)) x = b, optionally bordered, for R
// right-hand sides, in FP64 or FP32 with FP64 iterative refinement.
struct LinearProblem {
  Hier *h = nullptr;
  int R = 1;
  int border = 0;
  const double2 *shifts64 = nullptr;  // device, R (or null)
  const float2 *shifts32 = nullptr;   // device, R (or null)
};

static size_t solve_bytes(const Hier &h, int R, const heom_solver_opts &o) {
  const int64_t n = h.N * (int64_t)h.d * h.d;
  const bool flex = o.precond == HEOM_PREC_NN;
  const size_t v64 = (size_t)n * R * 16, v32 = (size_t)n * R * 8;
  size_t b = 0;
  if (o.mode == HEOM_SOLVE_FP32_IR) b = 2 * v64 + 2 * v32 + gmres_bytes(n, R, o.restart, flex, 8);
  else b = gmres_bytes(n, R, o.restart, flex, 16);
  b += (size_t)nchunk_for(n, R) * R * sizeof(double2) * 2 + R * sizeof(double2) * 4 + 4096;
  if (flex) b += nn_workspace_bytes(h, R, o.mode == HEOM_SOLVE_FP32_IR ? 8 : 16);
  return b;
}

template <typename T>
static std::function<heom_status(const void *, void *)> make_A(const LinearProblem &lp, hipStream_t s) {
  const int prec = std::is_same<T, double>::value ? HEOM_FP64 : HEOM_FP32;
  return [=](const void *in, void *out) -> heom_status {
    ApplyArgs a;
    a.x = in;
    a.y = out;
    a.n_rhs = lp.R;
    a.border = lp.border;
    a.shifts = std::is_same<T, double>::value ? (const void *)lp.shifts64 : (const void *)lp.shifts32;
    return launch_apply(*lp.h, prec, a, s);
  };
}

template <typename T>
static std::function<heom_status(const void *, void *, bool)> make_P(const LinearProblem &lp, const heom_solver_opts &o,
                                                                    NnApply *nn, hipStream_t s) {
  if (o.precond == HEOM_PREC_JACOBI || o.precond == HEOM_PREC_SCALED)
    return [=](const void *in, void *out, bool) -> heom_status {
      return jacobi<T>(in, out, *lp.h, lp.R, lp.shifts64, lp.border, s, o.precond == HEOM_PREC_SCALED);
    };
  if (o.precond == HEOM_PREC_BLOCK)
    return [=](const void *in, void *out, bool) -> heom_status {
      return block_prec<T>(in, out, *lp.h, lp.R, lp.shifts64, s);
    };
  if (o.precond == HEOM_PREC_NN && nn)
    return [=](const void *in, void *out, bool) -> heom_status { return nn->apply<T>(in, out, s); };
  return nullptr;
}

// Solve on [n][R] device vectors b (FP64) -> x (FP64, initial guess when
// x_given).  Fills the report; returns HEOM_ERR_NOT_CONVERGED when the true
// residual misses the tolerance.
static heom_status solve_system(const LinearProblem &lp, const heom_solver_opts &o, const void *b64, void *x64,
                                bool x_given, heom_solver_report *rep, WsArena &ws, hipStream_t s) {
  Hier &h = *lp.h;
  const int R = lp.R;
  const int64_t n = h.N * (int64_t)h.d * h.d;
  const int64_t nr = n * R;
  auto t0 = std::chrono::steady_clock::now();
  GmresStats st;
  NnApply nn;
  NnApply *nnp = nullptr;
  if (o.precond == HEOM_PREC_NN) {
    if (!o.nn) return fail(HEOM_ERR_ARG, "HEOM_PREC_NN needs opts.nn");
    HEOM_TRY(nn.init(o.nn, h, lp.R, lp.shifts64, lp.border, ws, o.mode == HEOM_SOLVE_FP32_IR ? 8 : 16));
    nnp = &nn;
  }
  const bool flex = nnp != nullptr;
  const int nch = nchunk_for(n, R);
  double2 *partial = (double2 *)ws.take((size_t)nch * R * sizeof(double2) * 2);
  double2 *hsm = (double2 *)ws.take(R * sizeof(double2) * 4);
  if (!partial || !hsm) return fail(HEOM_ERR_ARG, "solver workspace too small");
  PinnedBuf pin;
  std::vector<double> bn;
  HEOM_TRY(vec_norm<double>(b64, n, R, partial, nch, hsm, pin, bn, s));
  int refinements = 0;
  if (o.mode == HEOM_SOLVE_FP64) {
    Gmres<double> gm;
    HEOM_TRY(gm.init(ws, n, R, o.restart, flex));
    gm.A = make_A<double>(lp, s);
    gm.P = make_P<double>(lp, o, nnp, s);
    if (flex && o.fallback) gm.stall = 0.9;  // hand over to Jacobi early on stagnation
    gm.deflate = o.deflate;
    if (!x_given) HEOM_HIP_CHECK(hipMemsetAsync(x64, 0, sizeof(double2) * nr, s));
    HEOM_TRY(gm.solve((const double2 *)b64, (double2 *)x64, o.tol, o.max_iter, !x_given, st, s));
  } else {
    double2 *r64 = (double2 *)ws.take(sizeof(double2) * nr);
    float2 *r32 = (float2 *)ws.take(sizeof(float2) * nr);
    float2 *d32 = (float2 *)ws.take(sizeof(float2) * nr);
    if (!r64 || !r32 || !d32) return fail(HEOM_ERR_ARG, "solver workspace too small");
    Gmres<float> gm;
    HEOM_TRY(gm.init(ws, n, R, o.restart, flex));
    gm.deflate = o.deflate;
    gm.A = make_A<float>(lp, s);
    gm.P = make_P<float>(lp, o, nnp, s);
    auto A64 = make_A<double>(lp, s);
    if (!x_given) HEOM_HIP_CHECK(hipMemsetAsync(x64, 0, sizeof(double2) * nr, s));
    std::vector<double> rn;
    for (;; ++refinements) {
      HEOM_TRY(A64(x64, r64));
      ++st.applies;
      HEOM_TRY((axpby<double, double>(b64, 1.0, r64, -1.0, nr, s)));
      HEOM_TRY(vec_norm<double>(r64, n, R, partial, nch, hsm, pin, rn, s));
      double worst = 0, rmax = 0;
      for (int r = 0; r < R; ++r) {
        const double rel = bn[r] > 0 ? rn[r] / bn[r] : 0.0;
        if (!std::isfinite(rel)) return fail(HEOM_ERR_NAN, "non-finite residual in refinement");
        worst = std::max(worst, rel);
        rmax = std::max(rmax, rn[r]);
      }
      st.residual = worst;
      if (worst <= o.tol) { st.converged = true; break; }
      if (refinements >= o.max_refine || st.iterations >= o.max_iter) break;
      // one scale for all columns keeps the FP32 system linear in the columns
      const double sc = rmax > 0 ? 1.0 / rmax : 1.0;
      HEOM_TRY((axpby<double, float>(r64, sc, r32, 0.0, nr, s)));
      HEOM_HIP_CHECK(hipMemsetAsync(d32, 0, sizeof(float2) * nr, s));
      GmresStats inner;
      // each correction only needs a few digits: cap its iterations so a
      // stagnating FP32 solve hands back to the FP64 residual early
      const int cap = std::min(o.max_iter - st.iterations, std::max(4 * o.restart, 120));
      HEOM_TRY(gm.solve(r32, d32, o.inner_tol, cap, true, inner, s));
      st.iterations += inner.iterations;
      st.restarts += inner.restarts;
      st.applies += inner.applies;
      HEOM_TRY((axpby<float, double>(d32, 1.0 / sc, x64, 1.0, nr, s)));
    }
  }
  HEOM_HIP_CHECK(hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  if (rep) {
    rep->iterations += st.iterations;
    rep->restarts += st.restarts;
    rep->refinements += refinements;
    rep->applies += st.applies;
    rep->true_residual = std::max(rep->true_residual, st.residual);
    rep->seconds += std::chrono::duration<double>(t1 - t0).count();
    rep->fell_back = rep->fell_back || (nnp && nn.fell_back);
    rep->status = st.converged ? (rep->status ? rep->status : HEOM_OK) : HEOM_ERR_NOT_CONVERGED;
  }
  return st.converged ? HEOM_OK : fail(HEOM_ERR_NOT_CONVERGED, "solver did not reach the tolerance");
}

static heom_status check_opts(const heom_solver_opts *o) {
  if (!o) return fail(HEOM_ERR_ARG, "NULL options");
  if (o->restart < 1 || o->restart > 500) return fail(HEOM_ERR_ARG, "restart must be in [1, 500]");
  if (o->max_iter < 1) return fail(HEOM_ERR_ARG, "max_iter must be positive");
  if (!(o->tol > 0)) return fail(HEOM_ERR_ARG, "tol must be positive");
  if (o->mode != HEOM_SOLVE_FP64 && o->mode != HEOM_SOLVE_FP32_IR && o->mode != HEOM_SOLVE_SHIFTED)
    return fail(HEOM_ERR_ARG, "bad solve mode");
  if (o->mode == HEOM_SOLVE_SHIFTED && o->precond != HEOM_PREC_NONE)
    return fail(HEOM_ERR_ARG, "the multi-shift mode takes no preconditioner");
  if (o->precond < HEOM_PREC_NONE || o->precond > HEOM_PREC_BLOCK) return fail(HEOM_ERR_ARG, "bad preconditioner");
  if (o->deflate < 0 || o->deflate > kRotateMax - 1) return fail(HEOM_ERR_ARG, "deflate must be in [0, 31]");
  if (o->deflate > 0) {
    if (o->deflate + 2 > o->restart) return fail(HEOM_ERR_ARG, "deflate must be at most restart - 2");
    if (o->precond == HEOM_PREC_NN) return fail(HEOM_ERR_ARG, "deflated restarting needs a fixed preconditioner");
  }
  return HEOM_OK;
}

}  // namespace heom

using namespace heom;

extern "C" {

void heom_default_opts(heom_solver_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->restart = 30;
  o->max_iter = 3000;
  o->tol = 1e-8;
  o->precond = HEOM_PREC_JACOBI;
  o->mode = HEOM_SOLVE_FP64;
  o->inner_tol = 1e-5;
  o->max_refine = 20;
  o->rhs_chunk = 0;  // automatic (heom_spectrum_chunk)
  o->nn = nullptr;
  o->fallback = 1;
  o->use_x0 = 0;
}

// Frequencies per multi-RHS spectrum solve when rhs_chunk is 0: one for
// hierarchies of at least 2^18 elements per column (the one-column path
// works on whole blocks per wave and needs no column to wait for the slowest
// one), 16 below (launch latency dominates small systems).
static int auto_spectrum_chunk(const Hier &h) {
  const int64_t n = h.N * (int64_t)h.d * h.d;
  return n >= (int64_t(1) << 18) ? 1 : 16;
}

int32_t heom_spectrum_chunk(const heom_hier *hw, const heom_solver_opts *o) {
  if (!hw) return 0;
  if (o && o->rhs_chunk > 0) return o->rhs_chunk;
  return auto_spectrum_chunk(*hw->impl);
}

heom_status heom_workspace_size(const heom_hier *hw, int32_t op, const heom_solver_opts *o, int64_t n_rhs,
                                size_t *bytes) {
  if (!hw || !bytes) return fail(HEOM_ERR_ARG, "NULL argument");
  const Hier &h = *hw->impl;
  const int64_t n = h.N * (int64_t)h.d * h.d;
  if (op == HEOM_OP_PROPAGATE) {
    *bytes = 5 * (size_t)n * 16 + 4096;  // k1..k4 and the stage input at FP64 size (enough for FP32 too)
    return HEOM_OK;
  }
  heom_solver_opts d;
  if (!o) { heom_default_opts(&d); o = &d; }
  HEOM_TRY(check_opts(o));
  if (op == HEOM_OP_STEADY) {
    *bytes = (size_t)n * 16 + solve_bytes(h, 1, *o) + 4096;
    return HEOM_OK;
  }
  if (op == HEOM_OP_SPECTRUM && o->mode == HEOM_SOLVE_SHIFTED) {
    *bytes = shifted_bytes(h, *o) + 8192;
    return HEOM_OK;
  }
  if (op == HEOM_OP_SPECTRUM) {
    const int R = (int)std::max<int64_t>(1, n_rhs);
    *bytes = 2 * (size_t)n * R * 16 + solve_bytes(h, R, *o) + (size_t)R * 64 + 2 * (size_t)h.d * h.d * 16 + 8192;
    return HEOM_OK;
  }
  return fail(HEOM_ERR_ARG, "unknown workspace op");
}

static heom_status heom_propagate_body(heom_hier *hw, int32_t precision, void *x_dev, double dt, int64_t n_steps,
                           int64_t save_every, void *traj_dev, int32_t graph_steps, void *ws, size_t ws_bytes,
                           void *stream) {
  if (!hw || !x_dev || n_steps < 0 || !(std::isfinite(dt))) return fail(HEOM_ERR_ARG, "propagate: bad arguments");
  if (precision != HEOM_FP64 && precision != HEOM_FP32) return fail(HEOM_ERR_ARG, "bad precision");
  if (save_every < 0 || (save_every > 0 && !traj_dev)) return fail(HEOM_ERR_ARG, "propagate: bad trajectory args");
  Hier &h = *hw->impl;
  hipStream_t caller = (hipStream_t)stream;
  HEOM_TRY(ensure_device(h));
  if (rk4_small_fits(h)) {
    // small hierarchies: many whole steps per launch, in one workgroup
    const int64_t n_saves = save_every > 0 ? n_steps / save_every : 0;
    for (int64_t done = 0; done < n_steps; done += 4096)
      HEOM_TRY(launch_rk4_small(h, precision, x_dev, dt, std::min<int64_t>(4096, n_steps - done), save_every, done,
                                n_saves, traj_dev, caller));
    return HEOM_OK;
  }
  // Graph capture needs a non-default stream: run on a private stream that
  // is ordered after, and before, the caller's stream.
  const bool use_graph = graph_steps > 0 && n_steps >= graph_steps;
  hipStream_t s = caller;
  hipStream_t own = nullptr;
  hipEvent_t ev = nullptr;
  if (use_graph) {
    HEOM_HIP_CHECK(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    HEOM_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HEOM_HIP_CHECK(hipEventRecord(ev, caller));
    HEOM_HIP_CHECK(hipStreamWaitEvent(own, ev, 0));
    s = own;
  }
  struct Cleanup {
    hipStream_t own, caller;
    hipEvent_t ev;
    ~Cleanup() {
      if (own) {
        (void)hipEventRecord(ev, own);
        (void)hipStreamWaitEvent(caller, ev, 0);
        (void)hipStreamDestroy(own);
        (void)hipEventDestroy(ev);
      }
    }
  } cleanup{own, caller, ev};
  const int64_t n = h.N * (int64_t)h.d * h.d;
  const size_t w = precision == HEOM_FP64 ? 16 : 8;
  WsArena arena(ws, ws_bytes);
  void *k[4];
  for (int i = 0; i < 4; ++i) k[i] = arena.take((size_t)n * w);
  void *u = arena.take((size_t)n * w);  // stage input x + c k, formed once per stage
  int *counter = (int *)arena.take(256);
  if (!k[0] || !k[1] || !k[2] || !k[3] || !u || !counter) return fail(HEOM_ERR_ARG, "propagate: workspace too small");
  HEOM_TRY(fill_int(counter, 0, 1, s));
  const int64_t n_saves = save_every > 0 ? n_steps / save_every : 0;
  // Without Lindblad terms every stage's apply ends in an epilogue that
  // writes the next stage input u_s = x + c_s k_s (c_1 = c_2 = dt/2,
  // c_3 = dt) instead of k_s, and the last stage writes the new state over x.
  // With q = (u_1 + 2 u_2 - x) / 3, x + dt/6 (k_1 + 2 k_2 + 2 k_3 + k_4)
  // equals q + u_3 / 3 + dt/6 k_4.  The stages then read:
  //   1: u_1 = dt/2 (M + 2/dt) x             the shift supplies x, no extra read
  //   2: u_2 = x + dt/2 M u_1,  q = (x + u_1)/3 + dt/3 M u_1
  //                                          reads x and u_1 (the input's own
  //                                          block, mostly still in L2), writes q
  //   3: u_3 = x + dt M u_2                  reads x
  //   4: x <- q + dt/6 (M + 2/dt) u_3        reads q
  // so a step moves the four applies plus three vector reads and one write
  // beyond the stage outputs.  Stage 4 gathers only from u_3, and each
  // element of x is written by the lane that owns it, so the update is safe
  // in place.
  // (the shift 2/dt needs a step that is not vanishingly small)
  const bool fused = h.lind.empty() && std::fabs(dt) >= 1e-30;
  void *us[3] = {k[0], k[1], k[2]};
  void *q = k[3];
  auto fused_step = [&]() -> heom_status {
    ApplyArgs a;
    a.n_rhs = 1;
    a.epi = true;
    a.x = x_dev;
    a.y = us[0];
    a.eacc = 0.5 * dt;
    a.shift0 = 2.0 / dt;
    HEOM_TRY(launch_apply(h, precision, a, s));
    a = ApplyArgs{};
    a.n_rhs = 1;
    a.epi = true;
    a.x = us[0];
    a.y = us[1];
    a.ev[0] = x_dev;
    a.ev[1] = us[0];
    a.ec[0] = 1.0;
    a.eacc = 0.5 * dt;
    a.y2 = q;
    a.ec2[0] = 1.0 / 3.0;
    a.ec2[1] = 1.0 / 3.0;
    a.eacc2 = dt / 3.0;
    HEOM_TRY(launch_apply(h, precision, a, s));
    a = ApplyArgs{};
    a.n_rhs = 1;
    a.epi = true;
    a.x = us[1];
    a.y = us[2];
    a.ev[0] = x_dev;
    a.ec[0] = 1.0;
    a.eacc = dt;
    HEOM_TRY(launch_apply(h, precision, a, s));
    a = ApplyArgs{};
    a.n_rhs = 1;
    a.epi = true;
    a.x = us[2];
    a.y = x_dev;
    a.ev[0] = q;
    a.ec[0] = 1.0;
    a.eacc = dt / 6.0;
    a.shift0 = 2.0 / dt;
    return launch_apply(h, precision, a, s);
  };
  auto step = [&](int64_t idx) -> heom_status {
    if (fused) {
      HEOM_TRY(fused_step());
    } else {
      ApplyArgs a;
      a.n_rhs = 1;
      a.x = x_dev;
      a.y = k[0];
      HEOM_TRY(launch_apply(h, precision, a, s));
      const double cs[3] = {0.5 * dt, 0.5 * dt, dt};
      for (int st = 1; st < 4; ++st) {
        // one pass forms x + c k; the apply then gathers one block per
        // neighbour instead of two
        if (precision == HEOM_FP64) HEOM_TRY(stage_input<double>(x_dev, k[st - 1], cs[st - 1], u, n, s));
        else HEOM_TRY(stage_input<float>(x_dev, k[st - 1], cs[st - 1], u, n, s));
        a.x = u;
        a.y = k[st];
        HEOM_TRY(launch_apply(h, precision, a, s));
      }
      if (precision == HEOM_FP64) HEOM_TRY(rk4_combine<double>(x_dev, k[0], k[1], k[2], k[3], dt, n, s));
      else HEOM_TRY(rk4_combine<float>(x_dev, k[0], k[1], k[2], k[3], dt, n, s));
    }
    if (save_every > 0 && (idx + 1) % save_every == 0) {
      if (precision == HEOM_FP64) HEOM_TRY(save_rho0<double>(x_dev, traj_dev, h.d * h.d, counter, n_saves, s));
      else HEOM_TRY(save_rho0<float>(x_dev, traj_dev, h.d * h.d, counter, n_saves, s));
    }
    return HEOM_OK;
  };
  int64_t done = 0;
  if (use_graph) {
    if (save_every > 0 && graph_steps % save_every != 0)
      return fail(HEOM_ERR_ARG, "propagate: graph_steps must be a multiple of save_every");
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HEOM_HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    heom_status st = HEOM_OK;
    for (int i = 0; i < graph_steps && st == HEOM_OK; ++i) st = step(i);
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st != HEOM_OK) { if (graph) (void)hipGraphDestroy(graph); return st; }
    if (e != hipSuccess) return fail(HEOM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(HEOM_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    while (done + graph_steps <= n_steps) {
      e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) break;
      done += graph_steps;
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(HEOM_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  }
  for (; done < n_steps; ++done) HEOM_TRY(step(done));
  return HEOM_OK;
}

heom_status heom_propagate(heom_hier *hw, int32_t precision, void *x_dev, double dt, int64_t n_steps,
                           int64_t save_every, void *traj_dev, int32_t graph_steps, void *ws, size_t ws_bytes,
                           void *stream) {
  return guarded([&] { return heom_propagate_body(hw, precision, x_dev, dt, n_steps, save_every, traj_dev, graph_steps, ws, ws_bytes, stream); });
}

heom_status heom_steady_residual(heom_hier *hw, const void *x_dev, void *r_dev, void *stream) {
  if (!hw || !x_dev || !r_dev || x_dev == r_dev) return fail(HEOM_ERR_ARG, "steady_residual: bad arguments");
  Hier &h = *hw->impl;
  hipStream_t s = (hipStream_t)stream;
  ApplyArgs a;
  a.x = x_dev;
  a.y = r_dev;
  a.border = 1;
  HEOM_TRY(launch_apply(h, HEOM_FP64, a, s));
  const int64_t n = h.N * (int64_t)h.d * h.d;
  HEOM_TRY((axpby<double, double>(r_dev, 0.0, r_dev, -1.0, n, s)));
  HEOM_TRY(add_unit(r_dev, s));
  return HEOM_OK;
}

heom_status heom_vector_axpby(int32_t precision, const void *x_dev, double alpha, void *y_dev, double beta, int64_t n,
                              void *stream) {
  if (!x_dev || !y_dev || n < 0) return fail(HEOM_ERR_ARG, "vector_axpby: bad arguments");
  if (precision == HEOM_FP64) return axpby<double, double>(x_dev, alpha, y_dev, beta, n, (hipStream_t)stream);
  if (precision == HEOM_FP32) return axpby<float, float>(x_dev, alpha, y_dev, beta, n, (hipStream_t)stream);
  return fail(HEOM_ERR_ARG, "bad precision");
}

static heom_status heom_precondition_body(heom_hier *hw, int32_t precision, int32_t precond, const void *r_dev, void *z_dev,
                              int32_t n_rhs, const void *shifts_dev, int32_t border, void *stream) {
  if (!hw || !r_dev || !z_dev) return fail(HEOM_ERR_ARG, "precondition: NULL argument");
  if (r_dev == z_dev) return fail(HEOM_ERR_ARG, "precondition: r and z must not alias");
  if (n_rhs < 1) return fail(HEOM_ERR_ARG, "precondition: n_rhs must be positive");
  if (border && n_rhs != 1) return fail(HEOM_ERR_ARG, "precondition: border needs one right-hand side");
  if (precision != HEOM_FP64 && precision != HEOM_FP32) return fail(HEOM_ERR_ARG, "precondition: bad precision");
  if (precond != HEOM_PREC_JACOBI && precond != HEOM_PREC_SCALED && precond != HEOM_PREC_BLOCK)
    return fail(HEOM_ERR_ARG, "precondition: Jacobi, scaled or block only");
  Hier &h = *hw->impl;
  HEOM_TRY(ensure_device(h));
  hipStream_t s = (hipStream_t)stream;
  const double2 *sh = (const double2 *)shifts_dev;
  const bool fp64 = precision == HEOM_FP64;
  if (precond == HEOM_PREC_BLOCK)
    return fp64 ? block_prec<double>(r_dev, z_dev, h, n_rhs, sh, s) : block_prec<float>(r_dev, z_dev, h, n_rhs, sh, s);
  const int mod = precond == HEOM_PREC_SCALED;
  return fp64 ? jacobi<double>(r_dev, z_dev, h, n_rhs, sh, border, s, mod)
              : jacobi<float>(r_dev, z_dev, h, n_rhs, sh, border, s, mod);
}

heom_status heom_precondition(heom_hier *hw, int32_t precision, int32_t precond, const void *r_dev, void *z_dev,
                              int32_t n_rhs, const void *shifts_dev, int32_t border, void *stream) {
  return guarded([&] { return heom_precondition_body(hw, precision, precond, r_dev, z_dev, n_rhs, shifts_dev, border, stream); });
}

static heom_status heom_steady_body(heom_hier *hw, void *x_dev, const heom_solver_opts *o, heom_solver_report *r, void *ws,
                        size_t ws_bytes, void *stream) {
  if (!hw || !x_dev) return fail(HEOM_ERR_ARG, "steady: NULL argument");
  HEOM_TRY(check_opts(o));
  if (o->mode == HEOM_SOLVE_SHIFTED) return fail(HEOM_ERR_ARG, "steady: the multi-shift mode is for spectra");
  Hier &h = *hw->impl;
  if (h.parity != 1) return fail(HEOM_ERR_ARG, "steady: the stationary state lives in the even-parity hierarchy");
  hipStream_t s = (hipStream_t)stream;
  HEOM_TRY(ensure_device(h));
  if (r) std::memset(r, 0, sizeof(*r));
  const int64_t n = h.N * (int64_t)h.d * h.d;
  WsArena arena(ws, ws_bytes);
  double2 *b = (double2 *)arena.take(sizeof(double2) * n);
  if (!b) return fail(HEOM_ERR_ARG, "steady: workspace too small");
  // b = e_0: the bordered row (ADO 0, element (0,0)) carries Tr rho_0 = 1
  HEOM_HIP_CHECK(hipMemsetAsync(b, 0, sizeof(double2) * n, s));
  const double2 one = make_double2(1.0, 0.0);
  HEOM_HIP_CHECK(hipMemcpyAsync(b, &one, sizeof(double2), hipMemcpyHostToDevice, s));
  LinearProblem lp;
  lp.h = &h;
  lp.R = 1;
  lp.border = 1;
  heom_solver_report local;
  std::memset(&local, 0, sizeof(local));
  heom_solver_report *rp = r ? r : &local;
  heom_status st = solve_system(lp, *o, b, x_dev, o->use_x0 != 0, rp, arena, s);
  if ((st == HEOM_ERR_NOT_CONVERGED || st == HEOM_ERR_NAN) && o->precond == HEOM_PREC_NN && o->fallback) {
    // Jacobi GMRES takes over.  It continues from the network's iterate only
    // when that cut the residual tenfold: restarted GMRES started from a
    // barely improved iterate can stagnate where a zero start does not.
    heom_solver_opts o2 = *o;
    o2.precond = HEOM_PREC_JACOBI;
    o2.use_x0 = st != HEOM_ERR_NAN && rp->true_residual <= 0.1;
    // iterations, applies and seconds keep accumulating over both attempts
    rp->fell_back = 1;
    rp->status = HEOM_OK;
    rp->true_residual = 0.0;
    WsArena arena2(ws, ws_bytes);
    arena2.take(sizeof(double2) * n);
    st = solve_system(lp, o2, b, x_dev, o2.use_x0 != 0, rp, arena2, s);
  }
  return st;
}

heom_status heom_steady(heom_hier *hw, void *x_dev, const heom_solver_opts *o, heom_solver_report *r, void *ws,
                        size_t ws_bytes, void *stream) {
  return guarded([&] { return heom_steady_body(hw, x_dev, o, r, ws, ws_bytes, stream); });
}

static heom_status heom_spectrum_body(heom_hier *even, heom_hier *odd, const void *x_ss_dev, int32_t kind, const double *op,
                          const double *omega, int64_t n_omega, double *out_host, const heom_solver_opts *o,
                          heom_solver_report *r, void *ws, size_t ws_bytes, void *stream) {
  if (!even || !x_ss_dev || !op || !omega || !out_host || n_omega < 0) return fail(HEOM_ERR_ARG, "spectrum: NULL argument");
  HEOM_TRY(check_opts(o));
  if (kind != 0 && kind != 1) return fail(HEOM_ERR_ARG, "spectrum: kind must be 0 (DOS) or 1 (PSD)");
  if (o->deflate != 0 && o->mode != HEOM_SOLVE_SHIFTED)
    return fail(HEOM_ERR_UNSUPPORTED, "spectrum: thick restarts are for the multi-shift mode only");
  if (kind == 0 && !odd) return fail(HEOM_ERR_ARG, "spectrum: the density of states needs the odd-parity hierarchy");
  Hier &he = *even->impl;
  Hier &hs = kind == 0 ? *odd->impl : he;
  if (he.parity != 1 || (kind == 0 && hs.parity != -1)) return fail(HEOM_ERR_ARG, "spectrum: parity of the hierarchies");
  if (kind == 0 && (hs.N != he.N || hs.d != he.d)) return fail(HEOM_ERR_ARG, "spectrum: even and odd hierarchies differ");
  hipStream_t s = (hipStream_t)stream;
  HEOM_TRY(ensure_device(hs));
  if (r) std::memset(r, 0, sizeof(*r));
  if (o->mode == HEOM_SOLVE_SHIFTED)
    return spectrum_shifted(hs, (const double2 *)x_ss_dev, kind, op, omega, n_omega, out_host, *o, r, ws, ws_bytes, s);
  const int d = hs.d;
  const int64_t n = hs.N * (int64_t)d * d;
  const int per = kind == 0 ? 2 : 1;
  const int nw_chunk =
      (int)std::max<int64_t>(1, std::min<int64_t>(o->rhs_chunk > 0 ? o->rhs_chunk : auto_spectrum_chunk(hs), n_omega));
  const int Rmax = per * nw_chunk;
  WsArena arena(ws, ws_bytes);
  double2 *opsd = (double2 *)arena.take(2 * (size_t)d * d * sizeof(double2));
  int *colb = (int *)arena.take(Rmax * sizeof(int));
  int *colr = (int *)arena.take(Rmax * sizeof(int));
  double2 *sh64 = (double2 *)arena.take(Rmax * sizeof(double2));
  float2 *sh32 = (float2 *)arena.take(Rmax * sizeof(float2));
  double *outd = (double *)arena.take(Rmax * sizeof(double));
  double2 *b = (double2 *)arena.take((size_t)n * Rmax * sizeof(double2));
  double2 *x = (double2 *)arena.take((size_t)n * Rmax * sizeof(double2));
  if (!opsd || !colb || !colr || !sh64 || !sh32 || !outd || !b || !x)
    return fail(HEOM_ERR_ARG, "spectrum: workspace too small (see heom_workspace_size)");
  // ops[0] = op, ops[1] = op^dagger
  std::vector<double2> ops(2 * d * d);
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < d; ++k) {
      ops[i * d + k] = make_double2(op[2 * (i * d + k)], op[2 * (i * d + k) + 1]);
      ops[d * d + i * d + k] = make_double2(op[2 * (k * d + i)], -op[2 * (k * d + i) + 1]);
    }
  HEOM_HIP_CHECK(hipMemcpyAsync(opsd, ops.data(), ops.size() * sizeof(double2), hipMemcpyHostToDevice, s));
  std::vector<double> outh(Rmax);
  const size_t mark = arena.used;
  heom_status worst = HEOM_OK;
  for (int64_t w0 = 0; w0 < n_omega; w0 += nw_chunk) {
    const int nw = (int)std::min<int64_t>(nw_chunk, n_omega - w0);
    const int R = per * nw;
    std::vector<int> cb(R), cr(R);
    std::vector<double2> s64(R);
    std::vector<float2> s32(R);
    for (int q = 0; q < nw; ++q) {
      const double wq = omega[w0 + q];
      if (kind == 0) {
        // (M + i w) x_+ = op^dag rho  -> read Tr[op x_+];  (M - i w) x_- = op rho -> read Tr[op^dag x_-]
        cb[q] = 1; cr[q] = 0; s64[q] = make_double2(0.0, wq);
        cb[nw + q] = 0; cr[nw + q] = 1; s64[nw + q] = make_double2(0.0, -wq);
      } else {
        // (M - i w) x = op rho -> read Tr[op^dag x]
        cb[q] = 0; cr[q] = 1; s64[q] = make_double2(0.0, -wq);
      }
    }
    for (int q = 0; q < R; ++q) s32[q] = make_float2((float)s64[q].x, (float)s64[q].y);
    HEOM_HIP_CHECK(hipMemcpyAsync(colb, cb.data(), R * sizeof(int), hipMemcpyHostToDevice, s));
    HEOM_HIP_CHECK(hipMemcpyAsync(colr, cr.data(), R * sizeof(int), hipMemcpyHostToDevice, s));
    HEOM_HIP_CHECK(hipMemcpyAsync(sh64, s64.data(), R * sizeof(double2), hipMemcpyHostToDevice, s));
    HEOM_HIP_CHECK(hipMemcpyAsync(sh32, s32.data(), R * sizeof(float2), hipMemcpyHostToDevice, s));
    HEOM_TRY(left_multiply<double>((const double2 *)x_ss_dev, opsd, d, hs.N, R, colb, b, s));
    LinearProblem lp;
    lp.h = &hs;
    lp.R = R;
    lp.border = 0;
    lp.shifts64 = sh64;
    lp.shifts32 = sh32;
    arena.used = mark;
    const double res_before = r ? r->true_residual : 0.0;
    const int32_t status_before = r ? r->status : 0;
    heom_status st = solve_system(lp, *o, b, x, false, r, arena, s);
    if ((st == HEOM_ERR_NOT_CONVERGED || st == HEOM_ERR_NAN) && o->precond == HEOM_PREC_NN && o->fallback) {
      // Jacobi GMRES solves this chunk of frequencies again from zero; the
      // report keeps accumulating iterations, applies and seconds
      heom_solver_opts o2 = *o;
      o2.precond = HEOM_PREC_JACOBI;
      if (r) {
        r->fell_back = 1;
        r->true_residual = res_before;
        r->status = status_before;
      }
      arena.used = mark;
      st = solve_system(lp, o2, b, x, false, r, arena, s);
    }
    if (st != HEOM_OK && st != HEOM_ERR_NOT_CONVERGED) return st;
    if (st != HEOM_OK) worst = st;
    HEOM_TRY(trace_readout<double>(x, opsd, d, R, colr, -1.0 / kPi, outd, s));
    HEOM_HIP_CHECK(hipMemcpyAsync(outh.data(), outd, R * sizeof(double), hipMemcpyDeviceToHost, s));
    HEOM_HIP_CHECK(hipStreamSynchronize(s));
    for (int q = 0; q < nw; ++q) out_host[w0 + q] = kind == 0 ? outh[q] + outh[nw + q] : outh[q];
  }
  return worst == HEOM_OK ? HEOM_OK : fail(worst, "spectrum: some frequencies did not converge");
}

heom_status heom_spectrum(heom_hier *even, heom_hier *odd, const void *x_ss_dev, int32_t kind, const double *op,
                          const double *omega, int64_t n_omega, double *out_host, const heom_solver_opts *o,
                          heom_solver_report *r, void *ws, size_t ws_bytes, void *stream) {
  return guarded([&] { return heom_spectrum_body(even, odd, x_ss_dev, kind, op, omega, n_omega, out_host, o, r, ws, ws_bytes, stream); });
}

}  // extern "C"
