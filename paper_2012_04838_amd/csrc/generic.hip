// Host side of the general kernels (generic.hpp): the right-hand side and stage update, the
// statistics and the state conversions of plans whose N is not a power of two or that use
// the paper's phase-shift dealiasing.  N, K and the retained set come from the plan's
// geometry at run time; one schedule.
#include <type_traits>

#include "engine.hpp"
#include "generic.hpp"

namespace psdns {
namespace {

using gen::Factors;
using gen::Shape;
using gen::Spec;

// Output fields of the z inverse: U1 U2 U3 dzU1 dzU2, then Phi_s dzPhi_s (axis 3 = kz).
Spec z_inverse_spec(int S) {
  Spec s{};
  auto add = [&](int f, int axis) {
    const int o = s.nout++;
    s.nterm[o] = 1;
    s.f[o][0] = f;
    s.axis[o][0] = axis;
    s.sgn[o][0] = 1.f;
  };
  add(0, 0);
  add(1, 0);
  add(2, 0);
  add(0, 3);
  add(1, 3);
  for (int i = 0; i < S; ++i) {
    add(3 + i, 0);
    add(3 + i, 3);
  }
  return s;
}

// Output fields of the y inverse from the A fields (axis 2 = ky):
// u1 u2 u3, omega1 = dy u3 - dz u2, dz u1, dy u1, then phi_s, dy phi_s, dz phi_s.
Spec y_inverse_spec(int S) {
  Spec s{};
  auto add = [&](int f, int axis, float sg, int f2 = -1, int axis2 = 0, float sg2 = 0.f) {
    const int o = s.nout++;
    s.nterm[o] = f2 >= 0 ? 2 : 1;
    s.f[o][0] = f;
    s.axis[o][0] = axis;
    s.sgn[o][0] = sg;
    s.f[o][1] = f2 >= 0 ? f2 : 0;
    s.axis[o][1] = axis2;
    s.sgn[o][1] = sg2;
  };
  add(0, 0, 1.f);
  add(1, 0, 1.f);
  add(2, 0, 1.f);
  add(2, 2, 1.f, 4, 0, -1.f);
  add(3, 0, 1.f);
  add(0, 2, 1.f);
  for (int i = 0; i < S; ++i) {
    add(5 + 2 * i, 0, 1.f);
    add(5 + 2 * i, 2, 1.f);
    add(6 + 2 * i, 0, 1.f);
  }
  return s;
}

// Plain inverse of the first nf A fields (statistics).
Spec plain_spec(int nf) {
  Spec s{};
  for (int o = 0; o < nf; ++o) {
    s.nterm[o] = 1;
    s.f[o][0] = o;
    s.axis[o][0] = 0;
    s.sgn[o][0] = 1.f;
  }
  s.nout = nf;
  return s;
}

// fn(std::integral_constant<int, P>) for the runtime count p of positions per thread (1..16)
template <typename Fn>
void with_positions(int p, Fn&& fn) {
  switch (p) {
    case 1: fn(std::integral_constant<int, 1>{}); break;
    case 2: fn(std::integral_constant<int, 2>{}); break;
    case 3: fn(std::integral_constant<int, 3>{}); break;
    case 4: fn(std::integral_constant<int, 4>{}); break;
    case 5: fn(std::integral_constant<int, 5>{}); break;
    case 6: fn(std::integral_constant<int, 6>{}); break;
    case 7: fn(std::integral_constant<int, 7>{}); break;
    case 8: fn(std::integral_constant<int, 8>{}); break;
    case 9: fn(std::integral_constant<int, 9>{}); break;
    case 10: fn(std::integral_constant<int, 10>{}); break;
    case 11: fn(std::integral_constant<int, 11>{}); break;
    case 12: fn(std::integral_constant<int, 12>{}); break;
    case 13: fn(std::integral_constant<int, 13>{}); break;
    case 14: fn(std::integral_constant<int, 14>{}); break;
    case 15: fn(std::integral_constant<int, 15>{}); break;
    default: fn(std::integral_constant<int, 16>{}); break;
  }
}

template <typename T>
struct GEngine {
  static Shape shape(const Geom& g) { return gen::col_shape(g.N, (int)sizeof(cpx<T>)); }
  // x pass: P positions per lane of the physical fields, lw lines (wavefronts) per block
  template <int P>
  static void launch_x(const Ctx& x, int shift, int umax, hipStream_t s) {
    const Geom& g = x.g;
    const int csize = (int)sizeof(cpx<T>);
    const int lw = gen::x_lines(g.N, csize);
    const long long lines = (long long)g.N * g.N;
    gen::k_x_pass<T, P><<<dim3((unsigned)((lines + lw - 1) / lw), g.batch), 64 * lw, gen::x_lds_bytes(g.N, csize, lw),
                          s>>>(static_cast<cpx<T>*>(x.bbuf), static_cast<const cpx<T>*>(x.tw), x.slots, x.dyn, g,
                               gen::factor(g.N), shift, umax);
  }
  // the line-moment kernel of the statistics: up to 256 threads per line
  static int moment_threads(const Geom& g) {
    int t = 64;
    while (t < 256 && t < g.N / 2) t *= 2;
    return t;
  }

  static void z_inverse(const Ctx& x, const void* in, int shift, const Spec& sp, hipStream_t s) {
    const Geom& g = x.g;
    const Shape sh = shape(g);
    const cpx<T>* tw = static_cast<const cpx<T>*>(x.tw);
    const T scale = T(1) / (T(g.N) * T(g.N) * T(g.N));
    gen::k_z_inverse<T><<<dim3((g.KX + sh.W - 1) / sh.W, g.M, g.batch), sh.W * sh.TT, sh.lds, s>>>(
        static_cast<const cpx<T>*>(in), static_cast<cpx<T>*>(x.abuf), tw, x.slots, g, gen::factor(g.N), sp, sh.W,
        sh.TT, shift, scale);
  }
  static void y_inverse(const Ctx& x, int shift, const Spec& sp, hipStream_t s) {
    const Geom& g = x.g;
    const Shape sh = shape(g);
    gen::k_y_inverse<T><<<dim3((g.KX + sh.W - 1) / sh.W, g.N, g.batch), sh.W * sh.TT, sh.lds, s>>>(
        static_cast<const cpx<T>*>(x.abuf), static_cast<cpx<T>*>(x.bbuf), static_cast<const cpx<T>*>(x.tw), x.slots,
        g, gen::factor(g.N), sp, sh.W, sh.TT, shift);
  }
  static void x_pass(const Ctx& x, int shift, int umax, hipStream_t s) {
    with_positions(gen::x_positions(x.g.N), [&](auto p) { launch_x<decltype(p)::value>(x, shift, umax, s); });
  }
  static void y_forward(const Ctx& x, void* out, int out_fields, int shift, hipStream_t s) {
    const Geom& g = x.g;
    const Shape sh = shape(g);
    gen::k_y_forward<T><<<dim3((g.KX + sh.W - 1) / sh.W, g.N, g.batch), sh.W * sh.TT, sh.lds, s>>>(
        static_cast<const cpx<T>*>(x.bbuf), static_cast<cpx<T>*>(out), out_fields, static_cast<const cpx<T>*>(x.tw),
        x.slots, g, gen::factor(g.N), g.F, sh.W, sh.TT, shift);
  }

  // One evaluation of the right-hand side at stage_in and the update of `stage` (or dy/dt
  // into rhs_out for stage < 0).  With the sphere, the products are evaluated twice: on the
  // grid (kept in akeep) and on the shifted grid (in A); the z-forward pass takes the mean.
  static void rhs_stage(const Ctx& x, void* state, const void* stage_in, int stage, void* rhs_out, int want_max,
                        double dt_arg, int flags, hipStream_t s) {
    const Geom& g = x.g;
    const cpx<T>* sin = static_cast<const cpx<T>*>(stage_in);
    {
      TimedLaunch tl(x.timer, KID_FORCE, s);
      k_forcing_amplitude<T><<<g.batch, 256, 0, s>>>(sin, x.slots, x.dyn, g);
    }
    if (flags & kStagePrologue) return;
    const Spec zs = z_inverse_spec(g.S), ys = y_inverse_spec(g.S);
    const int passes = g.sphere ? 2 : 1;
    for (int p = 0; p < passes; ++p) {
      const int shift = p;  // the second evaluation is on the shifted grid
      {
        TimedLaunch tl(x.timer, KID_ZINV, s);
        z_inverse(x, stage_in, shift, zs, s);
      }
      {
        TimedLaunch tl(x.timer, KID_YINV, s);
        y_inverse(x, shift, ys, s);
      }
      {
        TimedLaunch tl(x.timer, KID_XPASS, s);
        // Eq. (10) takes the maximum over the grid points themselves: unshifted pass only
        x_pass(x, shift, want_max && p == 0, s);
      }
      if (stage == 0 && p == 0) {
        TimedLaunch tl(x.timer, KID_DT, s);
        k_step_dt<<<g.batch, 64, 0, s>>>(x.slots, x.dyn, g, dt_arg);
        k_stochastic_update<T><<<g.batch, 256, 0, s>>>(static_cast<const cpx<T>*>(state), x.slots, x.dyn, x.fband, g);
      }
      {
        TimedLaunch tl(x.timer, KID_YFWD, s);
        const bool keep = g.sphere && p == 0;
        y_forward(x, keep ? x.akeep : x.abuf, keep ? g.F : g.FA, shift, s);
      }
    }
    gen::GStage<T> sa;
    sa.yn = static_cast<cpx<T>*>(state);
    sa.acc = static_cast<cpx<T>*>(x.acc);
    sa.ys = static_cast<cpx<T>*>(x.ystage);
    sa.sin = sin;
    sa.rhs = static_cast<cpx<T>*>(rhs_out);
    sa.fband = x.fband;
    sa.stage = stage;
    TimedLaunch tl(x.timer, KID_ZFWD, s);
    with_positions(gen::zf_positions(g.N, gen::zf_shape(g.N, (int)sizeof(cpx<T>)).TT),
                   [&](auto p) { launch_zf<decltype(p)::value>(x, sa, s); });
  }
  // z forward + update: P positions per thread of each column
  template <int P>
  static void launch_zf(const Ctx& x, const gen::GStage<T>& sa, hipStream_t s) {
    const Geom& g = x.g;
    const Shape sh = gen::zf_shape(g.N, (int)sizeof(cpx<T>));
    gen::k_z_forward_update<T, P><<<dim3((g.KX + sh.W - 1) / sh.W, g.M, g.batch), sh.W * sh.TT, sh.lds, s>>>(
        static_cast<const cpx<T>*>(x.abuf), g.sphere ? static_cast<const cpx<T>*>(x.akeep) : nullptr, sa,
        static_cast<const cpx<T>*>(x.tw), x.slots, x.dyn, g, gen::factor(g.N), sh.W, sh.TT);
  }

  static void init_field(const Ctx& x, void* state, int slot, uint64_t seed, double kp, int kind, double energy,
                         hipStream_t s) {
    const Geom& g = x.g;
    const long long nmodes = (long long)g.M * g.M * g.KX;
    const int nb = (int)((nmodes + 255) / 256);
    TimedLaunch tl(x.timer, KID_AUX, s);
    k_init_energy<<<nb, 256, 0, s>>>(g, seed, kp, kind, x.part);
    k_init_scale<<<1, 256, 0, s>>>(x.part, nb, energy, g.N, x.dyn + slot);
    k_init_write<T><<<nb, 256, 0, s>>>(static_cast<cpx<T>*>(state), g, slot, seed, kp, kind, x.dyn + slot);
  }

  static void get_state(const Ctx& x, const void* state, int slot, void* canon, hipStream_t s) {
    const Geom& g = x.g;
    const long long ncan = (long long)g.F * g.N * g.N * (g.N / 2 + 1);
    TimedLaunch tl(x.timer, KID_AUX, s);
    k_fill_zero<T><<<(unsigned)((ncan + 255) / 256), 256, 0, s>>>(static_cast<cpx<T>*>(canon), ncan);
    const long long n = (long long)g.F * g.M * g.M * g.KX;
    k_convert<T, true><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
        const_cast<cpx<T>*>(static_cast<const cpx<T>*>(state)), static_cast<cpx<T>*>(canon), g, slot);
  }

  static void set_state(const Ctx& x, void* state, int slot, const void* canon, hipStream_t s) {
    const Geom& g = x.g;
    const long long n = (long long)g.F * g.M * g.M * g.KX;
    TimedLaunch tl(x.timer, KID_AUX, s);
    k_convert<T, false><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
        static_cast<cpx<T>*>(state), const_cast<cpx<T>*>(static_cast<const cpx<T>*>(canon)), g, slot);
  }

  static void zero_scalars(const Ctx& x, void* state, int slot, hipStream_t s) {
    const Geom& g = x.g;
    const long long n = (long long)g.S * g.st_field;
    if (n == 0) return;
    cpx<T>* p = static_cast<cpx<T>*>(state) + (long long)slot * g.F * g.st_field + 3 * g.st_field;
    TimedLaunch tl(x.timer, KID_AUX, s);
    k_fill_zero<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
  }

  static void band_hold(const Ctx& x, void* state, hipStream_t s) {
    TimedLaunch tl(x.timer, KID_FORCE, s);
    k_band_hold<T><<<x.g.batch, 256, 0, s>>>(static_cast<cpx<T>*>(state), x.slots, x.g);
  }

  // Spectra and statistics: shell sums on the state; moments through general z and y
  // inverses of the derivative fields and line transforms along x.
  static void spectra(const Ctx& x, const void* state, double* out, int flags, hipStream_t s) {
    const Geom& g = x.g;
    const int ns = g.ns, Q = shell_quantities(g.S);
    double* shells = x.stat;
    double* mom1 = shells + (long long)g.batch * ns * Q;
    double* mom2 = mom1 + (long long)g.batch * x.nbm * (3 * 6 + 1);
    TimedLaunch tl(x.timer, KID_AUX, s);
    const cpx<T>* st = static_cast<const cpx<T>*>(state);
    if (flags & 1) k_shell_sums<T><<<dim3(ns, g.batch), 256, 0, s>>>(st, x.slots, g, shells, ns);
    if (flags & 2) {
      const int t = moment_threads(g);
      const size_t xl = gen::moment_lds_bytes(g.N, (int)sizeof(cpx<T>), t);
      // first sweep: u1 u2 u3, du1/dx1, du2/dx2 (moments of the last two) and the max
      Spec z1{};
      const int f1[5] = {0, 1, 2, 0, 1}, a1[5] = {0, 0, 0, 1, 2};
      for (int i = 0; i < 5; ++i) {
        z1.nterm[i] = 1;
        z1.f[i][0] = f1[i];
        z1.axis[i][0] = a1[i];
        z1.sgn[i][0] = 1.f;
      }
      z1.nout = 5;
      z_inverse(x, state, 0, z1, s);
      y_inverse(x, 0, plain_spec(5), s);
      gen::k_x_moments<T><<<dim3(x.nbm, g.batch), t, xl, s>>>(static_cast<const cpx<T>*>(x.bbuf),
                                                             static_cast<const cpx<T>*>(x.tw), g, gen::factor(g.N), 5,
                                                             3, 1, mom1);
      // second sweep: du3/dx3, dphi_s/dx2
      Spec z2{};
      z2.nout = 1 + g.S;
      z2.nterm[0] = 1;
      z2.f[0][0] = 2;
      z2.axis[0][0] = 3;
      z2.sgn[0][0] = 1.f;
      for (int i = 0; i < g.S; ++i) {
        z2.nterm[1 + i] = 1;
        z2.f[1 + i][0] = 3 + i;
        z2.axis[1 + i][0] = 2;
        z2.sgn[1 + i][0] = 1.f;
      }
      z_inverse(x, state, 0, z2, s);
      y_inverse(x, 0, plain_spec(1 + g.S), s);
      gen::k_x_moments<T><<<dim3(x.nbm, g.batch), t, xl, s>>>(static_cast<const cpx<T>*>(x.bbuf),
                                                             static_cast<const cpx<T>*>(x.tw), g, gen::factor(g.N),
                                                             1 + g.S, 0, 0, mom2);
    }
    k_spectra_finalize<<<g.batch, 256, 0, s>>>(shells, mom1, mom2, x.nbm, x.slots, g, ns, flags, out, x.spectra_rec);
  }

  // dynamic LDS of the general kernels may exceed the default launch limit
  static void allow_lds() {
    const int b = 160 * 1024;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gen::k_z_inverse<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gen::k_y_inverse<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gen::k_y_forward<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b);
    for (int p = 1; p <= gen::kMaxPositions; ++p)
      with_positions(p, [&](auto q) {
        constexpr int P = decltype(q)::value;
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gen::k_x_pass<T, P>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, b);
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gen::k_z_forward_update<T, P>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, b);
      });
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gen::k_x_moments<T>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, b);
  }

  static Ops ops() {
    allow_lds();
    Ops o{};
    o.nsched = 1;
    StepSched& d = o.sched[0];
    d.ec = 0;
    d.ex = 0;
    d.col_w = 0;
    d.fused_ec = 0;
    d.fused_w = 0;
    d.x_lines = 1;
    d.rhs_stage = &rhs_stage;
    o.init_field = &init_field;
    o.get_state = &get_state;
    o.set_state = &set_state;
    o.spectra = &spectra;
    o.pressure = nullptr;
    o.band_hold = &band_hold;
    o.zero_scalars = &zero_scalars;
    return o;
  }
};

}  // namespace

Ops ops_general(int precision) { return precision == 32 ? GEngine<float>::ops() : GEngine<double>::ops(); }
int general_x_lines(int n, int precision) { return gen::x_lines(n, precision == 32 ? 8 : 16); }

}  // namespace psdns
