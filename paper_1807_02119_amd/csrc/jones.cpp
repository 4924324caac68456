// jones.cpp -- V_K(t(q)) = A(q) Z(q) (Eq. 4 of arXiv:1807.02119), plus t(q)
// (Eq. 1), status strings and the version string.
//
// With r the principal fourth root of t, t^{1/2} = r^2, t^{3/4} = r^3 and
// t^{tau/4} = r^tau.  Because (t^{1/2} + t^{-1/2})^2 = t + 2 + 1/t = q, the
// first base is -sqrt(q) for every supported q, so
//   log A = -(n_v+1) (log sqrt q + i pi) + w (3 log r + i pi) + tau log r.
// For q >= 4, t is real and positive (arg r = 0); for q = 2, 3, t = e^{i theta}
// with theta = pi/2, pi/3, so arg r = theta/4 is a rational multiple of pi and
// the phase of A is reduced exactly in integers before it is turned into an
// angle.
#include <cmath>

#include "internal.h"

namespace {

void t_of_q(int32_t q, double& re, double& im) {
  double qq = q;
  if (q < 4) {
    re = (qq - 2.0) / 2.0;
    im = std::sqrt(qq * (4.0 - qq)) / 2.0;
  } else {
    re = (qq - 2.0 + std::sqrt(qq * (qq - 4.0))) / 2.0;
    im = 0.0;
  }
}

}  // namespace

extern "C" kn_status kn_jones_variable(int32_t q, double* t_re, double* t_im) {
  if (q < 2 || q > 8) return KN_E_UNSUPPORTED;
  double re, im;
  t_of_q(q, re, im);
  if (t_re) *t_re = re;
  if (t_im) *t_im = im;
  return KN_OK;
}

extern "C" kn_status kn_jones(int32_t q, const kn_tait* g, const kn_scalar* z, double* v_re,
                              double* v_im, double* log2_abs_v, double* arg_v) {
  if (!g || !z) return KN_E_INVALID;
  if (q < 2 || q > 8) return KN_E_UNSUPPORTED;
  if (!std::isfinite(z->re) || !std::isfinite(z->im)) return KN_E_NUMERIC;
  const int64_t nv = g->n_vertices, w = g->writhe, tau = g->tau;
  if (z->re == 0.0 && z->im == 0.0) {
    if (v_re) *v_re = 0.0;
    if (v_im) *v_im = 0.0;
    if (log2_abs_v) *log2_abs_v = -INFINITY;
    if (arg_v) *arg_v = 0.0;
    return KN_OK;
  }
  double tr, ti;
  t_of_q(q, tr, ti);
  // |A| = q^{-(n_v+1)/2} |t|^{(3w+tau)/4}
  const int64_t k = 3 * w + tau;
  double log2_abs_t = (q < 4) ? 0.0 : std::log2(tr);
  double la = -0.5 * double(nv + 1) * std::log2((double)q) + 0.25 * double(k) * log2_abs_t;
  // arg A = pi (w - n_v - 1) + k arg(r), arg r = theta/4
  double argA;
  {
    int64_t pi_mult = ((w - nv - 1) % 2 + 2) % 2;  // 0 or 1 (times pi)
    // k * theta/4 as a multiple of pi: theta = pi/2 (q=2), pi/3 (q=3), 0 (q>=4)
    int64_t den = (q == 2) ? 8 : (q == 3) ? 12 : 0;
    double frac = 0.0;
    if (den) {
      int64_t num = ((k % (2 * den)) + 2 * den) % (2 * den);  // k/den pi mod 2 pi
      frac = double(num) / double(den);
    }
    double turns = double(pi_mult) + frac;  // in units of pi, in [0, 3)
    argA = M_PI * std::fmod(turns, 2.0);
  }
  // V = z * A: magnitude in log2, phase added
  double mz = std::hypot(z->re, z->im);
  double log2v = std::log2(mz) + double(z->exp2) + la;
  double argv = std::atan2(z->im, z->re) + argA;
  argv = std::remainder(argv, 2.0 * M_PI);
  if (log2_abs_v) *log2_abs_v = log2v;
  if (arg_v) *arg_v = argv;
  // complex value: split the exponent to keep the mantissa exact-ish
  double ei = std::floor(log2v);
  double mag = std::exp2(log2v - ei);
  double re = mag * std::cos(argv), im = mag * std::sin(argv);
  int e = ei > 4000 ? 4000 : (ei < -4000 ? -4000 : (int)ei);
  if (v_re) *v_re = std::ldexp(re, e);
  if (v_im) *v_im = std::ldexp(im, e);
  return KN_OK;
}

extern "C" const char* kn_status_string(kn_status s) {
  switch (s) {
    case KN_OK: return "ok";
    case KN_E_INVALID: return "invalid argument or diagram";
    case KN_E_NOMEM: return "out of host memory";
    case KN_E_BUDGET: return "plan exceeds the memory budget or workspace";
    case KN_E_DEVICE: return "HIP runtime error";
    case KN_E_NUMERIC: return "non-finite value";
    case KN_E_UNSUPPORTED: return "unsupported q or option combination";
  }
  return "unknown status";
}

extern "C" const char* kn_version(void) { return "kn 0.1 (gfx950)"; }
