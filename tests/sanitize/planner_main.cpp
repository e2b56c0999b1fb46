// Host planner of libxrd (xrd_batch_create and the host-only calls) under
// AddressSanitizer and UndefinedBehaviorSanitizer: plans batches of the
// workloads' shapes, invalid inputs, every structure-factor method, and
// checks a few plan invariants.  No HIP call is made (the device launch
// functions are replaced by stubs that abort if reached).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../include/xrd.h"

namespace {

int fails = 0;
void expect(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s (%s)\n", what, xrd_last_error());
    ++fails;
  }
}

struct Batch {
  std::vector<double> lat, tmin, tmax;
  std::vector<int64_t> off;
};

// n crystals: lengths U(lo, hi), angles U(60, 120) with the flatness test,
// atoms 1 .. max_atoms
Batch make(int n, double lo, double hi, int max_atoms, std::mt19937_64 &rng, double t0, double t1) {
  std::uniform_real_distribution<double> len(lo, hi), ang(60.0, 120.0);
  std::uniform_int_distribution<int> na(1, max_atoms);
  Batch b;
  b.off.push_back(0);
  for (int c = 0; c < n; ++c) {
    double al, be, ga;
    while (true) {
      al = ang(rng), be = ang(rng), ga = ang(rng);
      const double ca = std::cos(al * M_PI / 180), cb = std::cos(be * M_PI / 180), cg = std::cos(ga * M_PI / 180);
      if (1 - ca * ca - cb * cb - cg * cg + 2 * ca * cb * cg >= 1e-3) break;
    }
    b.lat.insert(b.lat.end(), {len(rng), len(rng), len(rng), al, be, ga});
    b.off.push_back(b.off.back() + na(rng));
    b.tmin.push_back(t0);
    b.tmax.push_back(t1);
  }
  return b;
}

xrd_batch_desc desc_of(const Batch &b, int precision, int friedel, int method, int forward_only) {
  xrd_batch_desc d{};
  d.n_crystals = (int64_t)b.tmin.size();
  d.n_species = 4;
  d.precision = precision;
  d.lattice = b.lat.data();
  d.atom_offset = b.off.data();
  d.two_theta_min = b.tmin.data();
  d.two_theta_max = b.tmax.data();
  d.wavelength = 1.54184;
  d.merge_tol = 1e-5;
  d.friedel = friedel;
  d.sf_method = method;
  d.forward_only = forward_only;
  // device pointers are never dereferenced by the planner
  static double fake[1];
  d.frac = d.occ = d.bfac = d.sf_coeff = fake;
  d.species = reinterpret_cast<const int32_t *>(fake);
  return d;
}

}  // namespace

int main() {
  std::mt19937_64 rng(12345);
  const Batch small = make(300, 3.0, 15.0, 200, rng, 10.0, 90.0);
  const Batch large = make(3, 25.0, 35.0, 3000, rng, 5.0, 120.0);
  for (const Batch *b : {&small, &large})
    for (int precision : {XRD_FP64, XRD_MIXED})
      for (int method : {XRD_SF_DIRECT, XRD_SF_RECURRENCE, XRD_SF_AUTO})
        for (int fo : {0, 1}) {
          xrd_batch_desc d = desc_of(*b, precision, precision == XRD_MIXED, method, fo);
          xrd_batch *h = nullptr;
          expect(xrd_batch_create(&d, &h) == XRD_OK && h, "create");
          xrd_sizes s{};
          expect(xrd_batch_sizes(h, &s) == XRD_OK, "sizes");
          expect(s.workspace_bytes > 0 && s.workspace_bytes % 256 == 0, "workspace size");
          expect(s.refl_capacity == 2 * s.half_capacity, "capacities");
          expect(s.noalloc_merge_bytes > 0 && s.noalloc_merge_bytes <= s.workspace_bytes, "merge scratch");
          xrd_batch_destroy(h);
        }
  // invalid inputs: every one refused with a message, nothing leaked
  {
    Batch b = make(4, 3.0, 6.0, 5, rng, 10.0, 90.0);
    xrd_batch *h = nullptr;
    xrd_batch_desc d = desc_of(b, XRD_MIXED, 1, XRD_SF_DIRECT, 0);
    d.merge_tol = 0.0;
    expect(xrd_batch_create(&d, &h) == XRD_ERR_INVALID_ARG && !h, "tolerance 0");
    d = desc_of(b, XRD_MIXED, 1, 7, 0);
    expect(xrd_batch_create(&d, &h) == XRD_ERR_INVALID_ARG && !h, "unknown method");
    b.lat[3] = b.lat[4] = b.lat[5] = 120.0;  // flat cell
    d = desc_of(b, XRD_MIXED, 1, XRD_SF_DIRECT, 0);
    expect(xrd_batch_create(&d, &h) == XRD_ERR_INVALID_CELL && !h, "flat cell");
    Batch c = make(2, 3.0, 6.0, 5, rng, 10.0, 90.0);
    c.off[1] = 7;
    c.off[2] = 3;  // decreasing offsets
    d = desc_of(c, XRD_MIXED, 1, XRD_SF_DIRECT, 0);
    expect(xrd_batch_create(&d, &h) == XRD_ERR_INVALID_ARG && !h, "decreasing offsets");
    Batch e = make(1, 800.0, 800.0, 1, rng, 10.0, 170.0);  // search box beyond the index range
    d = desc_of(e, XRD_MIXED, 1, XRD_SF_DIRECT, 0);
    expect(xrd_batch_create(&d, &h) == XRD_ERR_CAPACITY && !h, "box too large");
  }
  // an empty batch
  {
    Batch b;
    b.off.push_back(0);
    xrd_batch_desc d = desc_of(b, XRD_MIXED, 1, XRD_SF_AUTO, 0);
    xrd_batch *h = nullptr;
    expect(xrd_batch_create(&d, &h) == XRD_OK && h, "empty batch");
    xrd_batch_destroy(h);
  }
  std::printf("planner checks done, %d failures\n", fails);
  return fails == 0 ? 0 : 1;
}
