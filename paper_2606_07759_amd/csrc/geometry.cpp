// Host-side FP64 geometry: the composite affine map (paper Sec. 2.1) and the
// derivative maps of the plain misregistration parameters.
#include <cmath>
#include <cstring>

#include "common.hpp"

namespace {

// R(phi) = [[c, -s], [s, c]]; multiples of pi/2 (within 1e-12) are snapped to
// exact 0/+-1 so quarter turns are exact permutations.
void rot(double phi, double& c, double& s) {
  const double half_pi = 1.5707963267948966;
  double q = phi / half_pi;
  double qr = std::nearbyint(q);
  if (std::fabs(q - qr) < 1e-12) {
    long k = ((long)qr % 4 + 4) % 4;
    static const double cs[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    c = cs[k][0];
    s = cs[k][1];
  } else {
    c = std::cos(phi);
    s = std::sin(phi);
  }
}

// 3x3 affine (row-major, last row 0 0 1) helpers.
struct H3 {
  double m[3][3];
};

H3 h3(double a00, double a01, double a10, double a11, double t0, double t1) {
  H3 h{{{a00, a01, t0}, {a10, a11, t1}, {0, 0, 1}}};
  return h;
}

H3 mul(const H3& x, const H3& y) {
  H3 r{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += x.m[i][k] * y.m[k][j];
      r.m[i][j] = acc;
    }
  return r;
}

}  // namespace

extern "C" const char* synim_status_str(int status) {
  switch (status) {
    case SYNIM_OK: return "ok";
    case SYNIM_E_NULL: return "null pointer";
    case SYNIM_E_SHAPE: return "bad shape";
    case SYNIM_E_PARAM: return "bad parameter";
    case SYNIM_E_OOB: return "samples outside the IF grid";
    case SYNIM_E_WORKSPACE: return "workspace missing or too small";
    case SYNIM_E_HIP: return "HIP runtime error";
    case SYNIM_E_NOT_CONVERGED: return "not converged";
    case SYNIM_E_UNSUPPORTED: return "unsupported geometry";
    default: return "unknown status";
  }
}

extern "C" int synim_version(void) { return 10000; }

extern "C" int synim_affine_from_misreg(const synim_misreg* th, int H_in, int W_in, int H_out,
                                        int W_out, double kappa, synim_affine* A,
                                        synim_affine* dA) {
  if (!th || !A) return SYNIM_E_NULL;
  if (!(th->mag > 0) || !(kappa > 0) || H_in < 1 || W_in < 1 || H_out < 1 || W_out < 1)
    return SYNIM_E_PARAM;
  double c, s;
  rot(th->rot, c, s);
  // A = (kappa/m) R(-rho) = (kappa/m) [[c, s], [-s, c]]
  const double k = kappa / th->mag;
  const double a00 = k * c, a01 = k * s, a10 = -k * s, a11 = k * c;
  const double cox = 0.5 * (W_out - 1), coy = 0.5 * (H_out - 1);
  const double csx = 0.5 * (W_in - 1), csy = 0.5 * (H_in - 1);
  const double ctx = cox + th->shift_x, cty = coy + th->shift_y;
  A->A[0][0] = a00;
  A->A[0][1] = a01;
  A->A[1][0] = a10;
  A->A[1][1] = a11;
  A->b[0] = csx - (a00 * ctx + a01 * cty);
  A->b[1] = csy - (a10 * ctx + a11 * cty);
  if (dA) {
    // d/dt_x, d/dt_y: -(kappa/m) R(-rho) e
    std::memset(dA, 0, 4 * sizeof(synim_affine));
    dA[0].b[0] = -a00;
    dA[0].b[1] = -a10;
    dA[1].b[0] = -a01;
    dA[1].b[1] = -a11;
    // d/drho: -(kappa/m) R(-rho) J (p_o - c_o - t), J = [[0,-1],[1,0]]; A J = [[a01,-a00],[a11,-a10]]
    const double j00 = a01, j01 = -a00, j10 = a11, j11 = -a10;
    dA[2].A[0][0] = -j00;
    dA[2].A[0][1] = -j01;
    dA[2].A[1][0] = -j10;
    dA[2].A[1][1] = -j11;
    dA[2].b[0] = j00 * ctx + j01 * cty;
    dA[2].b[1] = j10 * ctx + j11 * cty;
    // d/dm: -(p_s - c_s)/m = -(A/m)(p_o - c_o - t)
    const double im = 1.0 / th->mag;
    dA[3].A[0][0] = -a00 * im;
    dA[3].A[0][1] = -a01 * im;
    dA[3].A[1][0] = -a10 * im;
    dA[3].A[1][1] = -a11 * im;
    dA[3].b[0] = (a00 * ctx + a01 * cty) * im;
    dA[3].b[1] = (a10 * ctx + a11 * cty) * im;
  }
  return SYNIM_OK;
}

extern "C" int synim_affine_from_geometry(const synim_geometry* g, int H_in, int W_in, int H_out,
                                          int W_out, synim_affine* A) {
  if (!g || !A) return SYNIM_E_NULL;
  if (H_in < 1 || W_in < 1 || H_out < 1 || W_out < 1) return SYNIM_E_PARAM;
  if (!(g->kappa > 0) || !(g->cone_scale > 0) || g->dm_mag == 0 || g->wfs_mag_x == 0 ||
      g->wfs_mag_y == 0)
    return SYNIM_E_PARAM;
  double c, s;
  rot(g->dm_rot, c, s);
  H3 dm = h3(g->dm_mag * c, -g->dm_mag * s, g->dm_mag * s, g->dm_mag * c, g->dm_shift_x,
             g->dm_shift_y);
  const double ic = 1.0 / (g->kappa * g->cone_scale);
  H3 cone = h3(ic, 0, 0, ic, -g->footprint_x * ic, -g->footprint_y * ic);
  rot(g->wfs_rot, c, s);
  H3 wfs = h3(g->wfs_mag_x * c, -g->wfs_mag_x * s, g->wfs_mag_y * s, g->wfs_mag_y * c,
              g->wfs_shift_x, g->wfs_shift_y);
  H3 F = mul(wfs, mul(cone, dm));
  // invert the forward affine: u = L^-1 (p - t)
  const double det = F.m[0][0] * F.m[1][1] - F.m[0][1] * F.m[1][0];
  if (!(std::fabs(det) > 0)) return SYNIM_E_PARAM;
  const double i00 = F.m[1][1] / det, i01 = -F.m[0][1] / det;
  const double i10 = -F.m[1][0] / det, i11 = F.m[0][0] / det;
  const double t0 = -(i00 * F.m[0][2] + i01 * F.m[1][2]);
  const double t1 = -(i10 * F.m[0][2] + i11 * F.m[1][2]);
  const double cox = 0.5 * (W_out - 1), coy = 0.5 * (H_out - 1);
  const double csx = 0.5 * (W_in - 1), csy = 0.5 * (H_in - 1);
  A->A[0][0] = i00;
  A->A[0][1] = i01;
  A->A[1][0] = i10;
  A->A[1][1] = i11;
  // p_s - c_s = M (p_o - c_o) + t
  A->b[0] = csx + t0 - (i00 * cox + i01 * coy);
  A->b[1] = csy + t1 - (i10 * cox + i11 * coy);
  return SYNIM_OK;
}

namespace synim {

int validate_wfs(const synim_wfs* wfs) {
  if (!wfs) return SYNIM_E_NULL;
  if (!wfs->valid_idx || !wfs->pupil) return SYNIM_E_NULL;
  if (wfs->n_sub_x < 1 || wfs->n_sub_y < 1 || wfs->p < 1 || wfs->p > 64 || wfs->n_valid < 1 ||
      (long)wfs->n_valid > (long)wfs->n_sub_x * wfs->n_sub_y)
    return SYNIM_E_SHAPE;
  if ((long)wfs->n_sub_x * wfs->p > 16384 || (long)wfs->n_sub_y * wfs->p > 16384)
    return SYNIM_E_SHAPE;
  return SYNIM_OK;
}

}  // namespace synim
