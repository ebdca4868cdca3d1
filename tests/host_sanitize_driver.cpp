// Host-side driver for the sanitizer test: runs the library's host geometry
// entry points on cases read from stdin, one per line, and prints each result
// with full precision.  Built with AddressSanitizer and UndefinedBehavior-
// Sanitizer (test infrastructure, not part of the library).
//   M sx sy rot mag H_in W_in H_out W_out kappa with_derivatives
//   G dm_sx dm_sy dm_rot dm_mag cone fp_x fp_y wfs_sx wfs_sy wfs_rot wfs_mx wfs_my kappa
//     H_in W_in H_out W_out
//   N              (null-pointer calls)
//   S status       (status string)
#include <cstdio>
#include <cstring>

#include "synim.h"

static void print_map(const synim_affine& A) {
  std::printf(" %.17g %.17g %.17g %.17g %.17g %.17g", A.A[0][0], A.A[0][1], A.A[1][0], A.A[1][1],
              A.b[0], A.b[1]);
}

int main() {
  char kind[4];
  while (std::scanf("%3s", kind) == 1) {
    if (std::strcmp(kind, "M") == 0) {
      synim_misreg th{};
      int hi, wi, ho, wo, der;
      double kappa;
      if (std::scanf("%lf %lf %lf %lf %d %d %d %d %lf %d", &th.shift_x, &th.shift_y, &th.rot,
                     &th.mag, &hi, &wi, &ho, &wo, &kappa, &der) != 10)
        return 2;
      synim_affine A{}, dA[4]{};
      const int rc = synim_affine_from_misreg(&th, hi, wi, ho, wo, kappa, &A, der ? dA : nullptr);
      std::printf("%d", rc);
      print_map(A);
      if (der)
        for (const auto& d : dA) print_map(d);
      std::printf("\n");
    } else if (std::strcmp(kind, "G") == 0) {
      synim_geometry g{};
      int hi, wi, ho, wo;
      if (std::scanf("%lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %d %d %d %d",
                     &g.dm_shift_x, &g.dm_shift_y, &g.dm_rot, &g.dm_mag, &g.cone_scale,
                     &g.footprint_x, &g.footprint_y, &g.wfs_shift_x, &g.wfs_shift_y, &g.wfs_rot,
                     &g.wfs_mag_x, &g.wfs_mag_y, &g.kappa, &hi, &wi, &ho, &wo) != 17)
        return 2;
      synim_affine A{};
      const int rc = synim_affine_from_geometry(&g, hi, wi, ho, wo, &A);
      std::printf("%d", rc);
      print_map(A);
      std::printf("\n");
    } else if (std::strcmp(kind, "N") == 0) {
      synim_misreg th{0, 0, 0, 1};
      synim_geometry g{};
      synim_affine A{};
      std::printf("%d %d %d %d\n", synim_affine_from_misreg(nullptr, 8, 8, 8, 8, 1.0, &A, nullptr),
                  synim_affine_from_misreg(&th, 8, 8, 8, 8, 1.0, nullptr, nullptr),
                  synim_affine_from_geometry(nullptr, 8, 8, 8, 8, &A),
                  synim_affine_from_geometry(&g, 8, 8, 8, 8, nullptr));
    } else if (std::strcmp(kind, "S") == 0) {
      int st;
      if (std::scanf("%d", &st) != 1) return 2;
      const char* s = synim_status_str(st);
      std::printf("%s\n", s ? s : "(null)");
    } else {
      return 2;
    }
  }
  return 0;
}
