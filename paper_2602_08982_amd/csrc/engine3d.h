// Full-3D kernel set for one (precision, lattice shape): launches of the
// kernels of kernels3d.h with the shape-dependent tiling.
#pragma once

#include "ctx.h"
#include "kernels3d_gen.h"

namespace tdslda {

// ----------------------------------------------------------------------------
// full-3D engine for one (precision, shape)
template <typename R, int NX, int NY, int NZ>
struct Engine3D final : Engine {
  using CFG = SlabCfg<NX, NY, NZ>;
  static constexpr int G = 32;     // states per density group
  static constexpr int TB1 = 64;   // lap1 block
  static constexpr int GTB = 64;   // line passes of the current, tau and B' (a lane pair per line) and of the field derivatives (a thread per line)
  // operator line passes (a lane pair per line): 256 threads, fewer where
  // the block's running sums (NL/2 samples per thread) would pass 64 KB
  static constexpr int NLMAX = NX > NY ? (NX > NZ ? NX : NZ) : (NY > NZ ? NY : NZ);
  static constexpr int OTB_FIT = int(65536 / ((NLMAX / 2) * sizeof(cpx<R>))) / kWave * kWave;
  static constexpr int OTB = OTB_FIT < 256 ? (OTB_FIT < kWave ? kWave : OTB_FIT) : 256;
  static constexpr int JG = sizeof(R) == 8 ? 256 : 128;  // states per group of the current / B' line passes
  static constexpr int M = NX * NY * NZ;
  static constexpr int NYZ = NY * NZ;
  int ngx() const override { return CFG::NGX; }
  int ncb() const override { return int(cdiv(NYZ, TB1)); }
  int group() const override { return G; }
  size_t elem_size() const override { return sizeof(cpx<R>); }

  double cx2(const Ctx& c) const { double k = 2 * kPi / (NX * c.lat.dx); return k * k; }
  double cy2(const Ctx& c) const { double k = 2 * kPi / (NY * c.lat.dy); return k * k; }
  double cz2(const Ctx& c) const { double k = 2 * kPi / (NZ * c.lat.dz); return k * k; }

  // general functional: rho, nu by the transform-free density pass and the
  // current j by one line pass per axis, both over groups of DG states
  void gen_dens(Ctx& c, const void* X, const double* scale, int64_t nst) {
    const unsigned ng = cdiv(nst, DG);
    c.launch(KC_DENS, [&] {
      hipLaunchKernelGGL((k_dens_sum<R, DG>), dim3(cdiv(M, DS_TB * DS_P), ng), dim3(DS_TB), 0, c.stream,
                         (const cpx<R>*)X, nst, int64_t(M), c.wu, c.wv, scale, c.dens_part);
    });
    jlines(c, X, scale, nst);
    c.nsg_used = int(ng);
  }
  // the current's group partials (groups of JG states) into c.jpart
  void jlines(Ctx& c, const void* X, const double* scale, int64_t nst) {
    const unsigned jg = cdiv(nst, JG);
    const cpx<R>* x = (const cpx<R>*)X;
    c.launch(KC_DENS, [&] {
      hipLaunchKernelGGL((k_jline<R, NX, NY, NZ, 0, GTB, JG>), dim3(cdiv(NYZ, GTB / 2), jg), dim3(GTB), 0, c.stream, x,
                         nst, scale, c.wu, c.wv, 2 * kPi / (NX * c.lat.dx), c.jpart);
    });
    c.launch(KC_DENS, [&] {
      hipLaunchKernelGGL((k_jline<R, NX, NY, NZ, 1, GTB, JG>), dim3(cdiv(NX * NZ, GTB / 2), jg), dim3(GTB), 0, c.stream,
                         x, nst, scale, c.wu, c.wv, 2 * kPi / (NY * c.lat.dy), c.jpart);
    });
    c.launch(KC_DENS, [&] {
      hipLaunchKernelGGL((k_jline<R, NX, NY, NZ, 2, GTB, JG>), dim3(cdiv(NX * NY, GTB / 2), jg), dim3(GTB), 0, c.stream,
                         x, nst, scale, c.wu, c.wv, 2 * kPi / (NZ * c.lat.dz), c.jpart);
    });
    c.njg_used = int(jg);
  }
  // general functional: H phi of every state into T (or out) by three line
  // passes; with hp the <H>_n partials go to the h slots after the NGX raw
  // slots (which the last pass clears)
  void gen_apply(Ctx& c, const void* X, const double* scale, double* hp, void* out, int64_t nst) {
    require(int(cdiv(NYZ, OTB / 2)) <= ncb(), TDSLDA_EINVAL, "internal: too few h slots for the x-line pass");
    const int64_t fcs = c.aslda ? M : 0;  // ASLDA: fields per spin
    const cpx<R>* x = (const cpx<R>*)X;
    cpx<R>* T = (cpx<R>*)c.T;
    const R *al = (const R*)c.hAl, *la = (const R*)c.hLa, *hA = (const R*)c.hA;
    const cpx<R>* hD = (const cpx<R>*)c.hD;
    constexpr int LPB = OTB / 2;  // lines per block
    // z first (contiguous lines: its T write is its only pass over T), then
    // y, then x with the local terms and <H>_n (coalesced lines)
    c.launch(KC_LAP1, [&] {
      hipLaunchKernelGGL((k_opline<R, NX, NY, NZ, 2, OTB, true, false>), dim3(cdiv(NX * NY, LPB), nst), dim3(OTB), 0,
                         c.stream, x, scale, T, nullptr, al, la, (const R*)c.hAz, hA, hD, nullptr, c.h_stride,
                         CFG::NGX, ncb(), 2 * kPi / (NZ * c.lat.dz), c.dV, fcs);
    });
    c.launch(KC_LAP1, [&] {
      hipLaunchKernelGGL((k_opline<R, NX, NY, NZ, 1, OTB, false, false>), dim3(cdiv(NX * NZ, LPB), nst), dim3(OTB), 0,
                         c.stream, x, scale, T, nullptr, al, la, (const R*)c.hAy, hA, hD, nullptr, c.h_stride,
                         CFG::NGX, ncb(), 2 * kPi / (NY * c.lat.dy), c.dV, fcs);
    });
    c.launch(KC_LAP1, [&] {
      hipLaunchKernelGGL((k_opline<R, NX, NY, NZ, 0, OTB, false, true>), dim3(cdiv(NYZ, LPB), nst), dim3(OTB), 0,
                         c.stream, x, scale, T, (cpx<R>*)out, al, la, (const R*)c.hAx, hA, hD, hp, c.h_stride,
                         CFG::NGX, ncb(), 2 * kPi / (NX * c.lat.dx), c.dV, fcs);
    });
  }
  // quantum friction: j and B' by line passes over state groups, div j by
  // line passes over the current field, N, then the dissipative fields
  void friction(Ctx& c, const void* X, const double* scale, int64_t nst) override {
    const unsigned ng = cdiv(nst, JG);
    const cpx<R>* x = (const cpx<R>*)X;
    const double kx = 2 * kPi / (NX * c.lat.dx), ky = 2 * kPi / (NY * c.lat.dy), kz = 2 * kPi / (NZ * c.lat.dz);
    jlines(c, X, scale, nst);
    c.launch(KC_FRICTION, [&] {
      hipLaunchKernelGGL((k_bpline<R, NX, NY, NZ, 0, GTB, JG>), dim3(cdiv(NYZ, GTB / 2), ng), dim3(GTB), 0, c.stream, x,
                         nst, scale, c.wu, c.wv, kx * kx, c.fric_part);
      hipLaunchKernelGGL((k_bpline<R, NX, NY, NZ, 1, GTB, JG>), dim3(cdiv(NX * NZ, GTB / 2), ng), dim3(GTB), 0, c.stream,
                         x, nst, scale, c.wu, c.wv, ky * ky, c.fric_part);
      hipLaunchKernelGGL((k_bpline<R, NX, NY, NZ, 2, GTB, JG>), dim3(cdiv(NX * NY, GTB / 2), ng), dim3(GTB), 0, c.stream,
                         x, nst, scale, c.wu, c.wv, kz * kz, c.fric_part);
      hipLaunchKernelGGL(k_fric_sum3d, dim3(cdiv(M, 256)), dim3(256), 0, c.stream, c.jpart, c.fric_part, int(ng),
                         int64_t(M), c.ainv, c.fric_j, c.fric_bp);
      hipLaunchKernelGGL((k_field_d1line<NX, NY, NZ, 0, GTB>), dim3(cdiv(NYZ, GTB)), dim3(GTB), 0, c.stream,
                         c.fric_j, kx, c.fric_div);
      hipLaunchKernelGGL((k_field_d1line<NX, NY, NZ, 1, GTB>), dim3(cdiv(NX * NZ, GTB)), dim3(GTB), 0, c.stream,
                         c.fric_j, ky, c.fric_div);
      hipLaunchKernelGGL((k_field_d1line<NX, NY, NZ, 2, GTB>), dim3(cdiv(NX * NY, GTB)), dim3(GTB), 0, c.stream,
                         c.fric_j, kz, c.fric_div);
      hipLaunchKernelGGL(k_sum_N, dim3(1), dim3(1024), 0, c.stream, int64_t(M), c.rho, c.dVe, c.fric_N);
      hipLaunchKernelGGL((k_fric3d_fields<R>), dim3(cdiv(M, 256)), dim3(256), 0, c.stream, int64_t(M), c.fric_div,
                         c.fric_bp, c.fric_N, c.nu, c.U, c.delta, c.vext, c.dext, c.fun.mu, c.f_alpha, c.f_beta,
                         c.f_gamma, c.f_rho0, c.f_Nreq, (R*)c.hA, (cpx<R>*)c.hD);
    });
  }
  // spin-imbalanced ASLDA: spin-resolved rho, nu (transform-free) and tau,
  // j by one line pass per axis, all over groups of DG states
  void aslda_dens(Ctx& c, const void* X, const double* scale, int64_t nst) {
    const unsigned ng = cdiv(nst, DG);
    const cpx<R>* x = (const cpx<R>*)X;
    const double kx = 2 * kPi / (NX * c.lat.dx), ky = 2 * kPi / (NY * c.lat.dy), kz = 2 * kPi / (NZ * c.lat.dz);
    const double px = kPi / c.lat.dx, py = kPi / c.lat.dy, pz = kPi / c.lat.dz;
    c.launch(KC_DENS, [&] {
      hipLaunchKernelGGL((k_dens_sum<R, DG, DS_P, 12, true>), dim3(cdiv(M, DS_TB * DS_P), ng), dim3(DS_TB), 0,
                         c.stream, x, nst, int64_t(M), c.wu, c.wv, scale, c.dens_part);
      hipLaunchKernelGGL((k_taujline<R, NX, NY, NZ, 0, GTB, DG>), dim3(cdiv(NYZ, GTB / 2), ng), dim3(GTB), 0, c.stream,
                         x, nst, scale, c.wu, c.wv, kx, px * px, c.dens_part);
      hipLaunchKernelGGL((k_taujline<R, NX, NY, NZ, 1, GTB, DG>), dim3(cdiv(NX * NZ, GTB / 2), ng), dim3(GTB), 0,
                         c.stream, x, nst, scale, c.wu, c.wv, ky, py * py, c.dens_part);
      hipLaunchKernelGGL((k_taujline<R, NX, NY, NZ, 2, GTB, DG>), dim3(cdiv(NX * NY, GTB / 2), ng), dim3(GTB), 0,
                         c.stream, x, nst, scale, c.wu, c.wv, kz, pz * pz, c.dens_part);
    });
    c.nsg_used = int(ng);
  }
  void dens(Ctx& c, const void* X, const double* scale, int64_t nst) override {
    if (c.aslda) {
      aslda_dens(c, X, scale, nst);
      return;
    }
    if (c.gen) {
      gen_dens(c, X, scale, nst);
      return;
    }
    dim3 grid(CFG::NGX, cdiv(nst, G));
    c.launch(KC_DENS_KIN, [&] {
      hipLaunchKernelGGL((k_dens<R, NX, NY, NZ, G>), grid, dim3(CFG::TB), 0, c.stream,
                         (const cpx<R>*)X, nst, c.wu, c.wv, c.scalars(const_cast<double*>(scale)),
                         c.dens_part, cy2(c), cz2(c), c.dV);
    });
    c.nsg_used = int(cdiv(nst, G));
  }
  // states per dens_sum group (FP64: 256 measured 12% faster than 64 at 32^3)
  static constexpr int DG = sizeof(R) == 8 ? 256 : 128;
  void dens_sum(Ctx& c, const void* X, const double* scale, int64_t nst) override {
    if (c.aslda) {
      aslda_dens(c, X, scale, nst);
      return;
    }
    if (c.gen) {
      gen_dens(c, X, scale, nst);
      return;
    }
    dim3 grid(cdiv(M, DS_TB * DS_P), cdiv(nst, DG));
    c.launch(KC_DENS, [&] {
      hipLaunchKernelGGL((k_dens_sum<R, DG>), grid, dim3(DS_TB), 0, c.stream, (const cpx<R>*)X, nst,
                         int64_t(M), c.wu, c.wv, scale, c.dens_part);
    });
    c.nsg_used = int(cdiv(nst, DG));
  }
  bool producer_kinetic() const override { return true; }
  int raw_h_slots() const override { return CFG::NGX; }
  void reduce_pot(Ctx& c, bool update) override {
    FunParams fp{c.fun.functional, c.fun.B, c.fun.C, c.fun.inv_g_bdg, c.fun.mu, c.ainv, c.dext};
    if (c.aslda) {
      c.launch(KC_REDUCE_POT, [&] {
        hipLaunchKernelGGL((k_reduce_aslda3d<R>), dim3(cdiv(M, 256)), dim3(256), 0, c.stream, c.dens_part,
                           c.nsg_used, int64_t(M), fp, c.fun.mu_b, c.lam, c.vext, c.rho, c.tau, c.nu, c.jc, c.U,
                           c.delta, (R*)c.hA, (cpx<R>*)c.hD, (R*)c.hAx, (R*)c.hAy, (R*)c.hAz, c.gscratch, int(update));
        if (update)  // alpha_s and its Laplacian (Eq. kinop-alpha) for each spin
          for (int sp = 0; sp < 2; ++sp)
            hipLaunchKernelGGL((k_field_lap3d<R>), dim3(cdiv(M, 256)), dim3(256), 0, c.stream, NX, NY, NZ,
                               c.gscratch + sp * M, c.circ, c.circ + NX, c.circ + NX + NY, (R*)c.hAl + sp * M,
                               (R*)c.hLa + sp * M);
      });
      return;
    }
    if (c.gen) {
      c.launch(KC_REDUCE_POT, [&] {
        hipLaunchKernelGGL((k_reduce_gen3d<R>), dim3(cdiv(M, 256)), dim3(256), 0, c.stream, c.dens_part, c.jpart,
                           c.nsg_used, c.njg_used, int64_t(M), fp, c.fun.A, c.lam, c.vext, c.rho, c.nu, c.jc, c.U, c.delta,
                           (R*)c.hA, (cpx<R>*)c.hD, (R*)c.hAx, (R*)c.hAy, (R*)c.hAz,
                           int(update && c.fun.functional == TDSLDA_FUNC_SLDA));
      });
      return;
    }
    c.launch(KC_REDUCE_POT, [&] {
      hipLaunchKernelGGL((k_reduce_pot<R>), dim3(cdiv(M, 256)), dim3(256), 0, c.stream, c.dens_part,
                         c.nsg_used, int64_t(M), fp, c.lam, c.vext, c.rho, c.nu, c.U, c.delta, (R*)c.hA,
                         (cpx<R>*)c.hD, int(update));
    });
  }
  void lap1(Ctx& c, const void* X, const double* scale, bool hpart, int64_t nst) override {
    if (c.gen) {  // the whole H phi into T (the evaluation's lap2 is then pointwise)
      gen_apply(c, X, scale, hpart ? c.h_part : nullptr, nullptr, nst);
      return;
    }
    dim3 grid(cdiv(NYZ, TB1), nst);
    c.launch(KC_LAP1, [&] {
      hipLaunchKernelGGL((k_lap1<R, NX, NYZ, TB1>), grid, dim3(TB1), 0, c.stream, (const cpx<R>*)X,
                         scale, (cpx<R>*)c.T, (const R*)c.hA, (const cpx<R>*)c.hD,
                         hpart ? c.h_part : nullptr, c.h_stride, CFG::NGX, cx2(c), c.dV);
    });
  }
  void lap2(Ctx& c, const L2Desc& d, int64_t nst) override {
    Lap2Args<R> A{};
    A.X = (const cpx<R>*)d.X;
    A.Xout = (cpx<R>*)d.Xout;
    A.T = (const cpx<R>*)d.T;
    A.hA = (const R*)c.hA;
    A.hD = (const cpx<R>*)c.hD;
    A.scale = d.scale;
    A.hshift = d.hshift;
    A.out = (cpx<R>*)d.out;
    A.acc = (cpx<R>*)d.acc;
    for (int i = 0; i < 5; ++i) A.hist[i] = (const cpx<R>*)d.hist[i];
    A.cout = (cpx<R>*)d.cout;
    A.nrm_part = d.nrm_part;
    A.nrm_stride = c.nrm_stride;
    A.np = c.np;
    A.nq = c.nq;
    for (int i = 0; i < 5; ++i) {
      A.b[i] = c.bco[i];
      A.a[i] = c.aco[i];
    }
    A.tay_re = d.tay_re;
    A.tay_im = d.tay_im;
    A.init_acc = d.init_acc;
    A.cy2 = cy2(c);
    A.cz2 = cz2(c);
    A.h_part = c.h_part;
    A.h_stride = c.h_stride;
    A.dV = c.dV;
    dim3 grid(CFG::NGX, nst), block(CFG::TB);
    if (c.gen) {  // T holds H phi (lap1): the integrator arithmetic only
      switch (d.mode) {
        case L2_H:
          c.launch(KC_LAP2_H, [&] { hipLaunchKernelGGL((k_pw_gen<R, NX, NY, NZ, L2_H>), grid, block, 0, c.stream, A); });
          break;
        case L2_F:
          c.launch(KC_LAP2_F, [&] { hipLaunchKernelGGL((k_pw_gen<R, NX, NY, NZ, L2_F>), grid, block, 0, c.stream, A); });
          break;
        case L2_CORR:
          c.launch(KC_LAP2_CORR, [&] { hipLaunchKernelGGL((k_pw_gen<R, NX, NY, NZ, L2_CORR>), grid, block, 0, c.stream, A); });
          break;
        case L2_FULL:
          c.launch(KC_LAP2_FULL, [&] {
            if (c.np == 3)
              hipLaunchKernelGGL((k_pw_gen<R, NX, NY, NZ, L2_FULL, 3, 4>), grid, block, 0, c.stream, A);
            else if (c.np == 5)
              hipLaunchKernelGGL((k_pw_gen<R, NX, NY, NZ, L2_FULL, 5, 5>), grid, block, 0, c.stream, A);
            else
              hipLaunchKernelGGL((k_pw_gen<R, NX, NY, NZ, L2_FULL, 4, 5>), grid, block, 0, c.stream, A);
          });
          break;
        default:
          c.launch(KC_LAP2_TAYLOR, [&] { hipLaunchKernelGGL((k_pw_gen<R, NX, NY, NZ, L2_TAYLOR>), grid, block, 0, c.stream, A); });
      }
      return;
    }
    switch (d.mode) {
      case L2_H:
        c.launch(KC_LAP2_H, [&] { hipLaunchKernelGGL((k_lap2<R, NX, NY, NZ, L2_H>), grid, block, 0, c.stream, A); });
        break;
      case L2_F:
        c.launch(KC_LAP2_F, [&] { hipLaunchKernelGGL((k_lap2<R, NX, NY, NZ, L2_F>), grid, block, 0, c.stream, A); });
        break;
      case L2_CORR:
        c.launch(KC_LAP2_CORR, [&] { hipLaunchKernelGGL((k_lap2<R, NX, NY, NZ, L2_CORR>), grid, block, 0, c.stream, A); });
        break;
      case L2_FULL:
        c.launch(KC_LAP2_FULL, [&] {
          if (c.np == 3)
            hipLaunchKernelGGL((k_lap2<R, NX, NY, NZ, L2_FULL, 3, 4>), grid, block, 0, c.stream, A);
          else if (c.np == 5)
            hipLaunchKernelGGL((k_lap2<R, NX, NY, NZ, L2_FULL, 5, 5>), grid, block, 0, c.stream, A);
          else
            hipLaunchKernelGGL((k_lap2<R, NX, NY, NZ, L2_FULL, 4, 5>), grid, block, 0, c.stream, A);
        });
        break;
      default:
        c.launch(KC_LAP2_TAYLOR, [&] { hipLaunchKernelGGL((k_lap2<R, NX, NY, NZ, L2_TAYLOR>), grid, block, 0, c.stream, A); });
    }
  }
  void pointwise(Ctx& c, const PwDesc& d, int64_t nst) override {
    PwArgs<R> A{};
    A.X = (cpx<R>*)d.X;
    A.scale = d.scale;
    for (int i = 0; i < 5; ++i) A.hist[i] = (const cpx<R>*)d.hist[i];
    A.cout = (cpx<R>*)d.cout;
    A.nrm_part = d.nrm_part;
    A.nrm_stride = c.nrm_stride;
    A.np = c.np;
    A.nq = c.nq;
    for (int i = 0; i < 5; ++i) {
      A.b[i] = c.bco[i];
      A.a[i] = c.aco[i];
    }
    A.out64 = (cpx<double>*)d.out64;
    A.nst = nst;
    dim3 grid(CFG::NGX, state_rows(nst)), block(CFG::TB);
    if (d.mode == PW_NORM)
      c.launch(KC_NORM, [&] { hipLaunchKernelGGL((k_pointwise<R, NX, NY, NZ, PW_NORM>), grid, block, 0, c.stream, A); });
    else if (d.mode == PW_PRED)
      c.launch(KC_PRED, [&] {
        if (c.np == 3)
          hipLaunchKernelGGL((k_pointwise<R, NX, NY, NZ, PW_PRED, 3, 4>), grid, block, 0, c.stream, A);
        else if (c.np == 5)
          hipLaunchKernelGGL((k_pointwise<R, NX, NY, NZ, PW_PRED, 5, 5>), grid, block, 0, c.stream, A);
        else
          hipLaunchKernelGGL((k_pointwise<R, NX, NY, NZ, PW_PRED, 4, 5>), grid, block, 0, c.stream, A);
      });
    else
      c.launch(KC_SETUP, [&] { hipLaunchKernelGGL((k_pointwise<R, NX, NY, NZ, PW_SCALE>), grid, block, 0, c.stream, A); });
  }
  void grad(Ctx& c, const void* X, const double* scale, int64_t n0, int64_t nchunk) override {
    constexpr int TBG = 64;
    double* ts = c.gscratch;
    double* js = c.gscratch + nchunk * M;
    const double px = kPi / c.lat.dx, py = kPi / c.lat.dy, pz = kPi / c.lat.dz;
    c.launch(KC_GRAD, [&] {
      hipLaunchKernelGGL((k_grad_axis<R, NX, 0, TBG>), dim3(cdiv(M / NX, TBG), nchunk), dim3(TBG), 0,
                         c.stream, (const cpx<R>*)X, n0, nchunk, int64_t(M), int64_t(NYZ), int64_t(NYZ),
                         scale, c.wu, c.wv, 2 * kPi / (NX * c.lat.dx), px * px, ts, js);
    });
    c.launch(KC_GRAD, [&] {
      hipLaunchKernelGGL((k_grad_axis<R, NY, 1, TBG>), dim3(cdiv(M / NY, TBG), nchunk), dim3(TBG), 0,
                         c.stream, (const cpx<R>*)X, n0, nchunk, int64_t(M), int64_t(NZ), int64_t(NZ),
                         scale, c.wu, c.wv, 2 * kPi / (NY * c.lat.dy), py * py, ts, js);
    });
    c.launch(KC_GRAD, [&] {
      hipLaunchKernelGGL((k_grad_axis<R, NZ, 2, TBG>), dim3(cdiv(M / NZ, TBG), nchunk), dim3(TBG), 0,
                         c.stream, (const cpx<R>*)X, n0, nchunk, int64_t(M), int64_t(1), int64_t(1),
                         scale, c.wu, c.wv, 2 * kPi / (NZ * c.lat.dz), pz * pz, ts, js);
    });
  }
};

}  // namespace tdslda
