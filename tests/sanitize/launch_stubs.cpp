// Stand-ins for the device launch functions of libxrd, for host-only builds
// of the planner: the host calls exercised there never launch, so each stub
// aborts if reached.
#include <cstdio>
#include <cstdlib>

#include "xrd_internal.h"

namespace {
[[noreturn]] void reached(const char *name) {
  std::fprintf(stderr, "device launch %s reached in a host-only build\n", name);
  std::abort();
}
}  // namespace

namespace xrd {
void launch_fill_i32(int32_t *, int64_t, int32_t, hipStream_t) { reached("fill_i32"); }
void launch_fill_u64(uint64_t *, int64_t, uint64_t, hipStream_t) { reached("fill_u64"); }
hipError_t noalloc_scratch(void **) { reached("noalloc_scratch"); }
void launch_scan_i32(const int32_t *, int64_t, const int64_t *, int64_t *, int64_t *, hipStream_t) { reached("scan"); }
void launch_peak_families(const HChunk *, int64_t, const FamOps *, const int64_t *, const int64_t *, const int32_t *,
                          const int64_t *, const int16_t *, const int16_t *, const int16_t *, int, int32_t *,
                          int32_t *, int64_t *, int32_t *, hipStream_t) {
  reached("families");
}
void launch_enumerate(const CrystalPlan *, int64_t, const EnumChunk *, int64_t, double, int32_t *, int64_t *,
                      int64_t *, int16_t *, int16_t *, int16_t *, double *, double *, double *, int64_t *, int32_t,
                      const double *, const int32_t *, const double *, const double *, const double *, CoeffF *,
                      AtomRec *, AtomRot *, int32_t *, SpeciesRun *, int32_t *, int32_t *, int64_t, int64_t, hipStream_t) {
  reached("enumerate");
}
void launch_sf(bool, bool, const SfItem *, int64_t, int64_t, const CrystalPlan *, const int64_t *, const int16_t *,
               const int16_t *, const int16_t *, const double *, const double *, const AtomRec *, const SpeciesRun *,
               const int32_t *, const double *, const CoeffF *, void *, void *, double *, void *, int, hipStream_t) {
  reached("sf");
}
void launch_sf_rec(bool, bool, const SfRecArgs &, void *, void *, double *, void *, hipStream_t) { reached("sf_rec"); }
void launch_sort(const SortArgs &, hipStream_t) { reached("sort"); }
void launch_combine_lines(int64_t, const LinePeaks &, const LinePeaks *, const LineOut &, hipStream_t) {
  reached("combine_lines");
}
void launch_merge(const MergeArgs &, hipStream_t) { reached("merge"); }
void launch_broaden_fwd(bool, const HChunk *, int64_t, const CrystalPlan *, const int32_t *, int64_t, bool,
                        const int64_t *, const double *, const int32_t *, const double *, double, double, int64_t,
                        double, double, int64_t, double *, int32_t *, int32_t *, double *, hipStream_t) {
  reached("broaden_fwd");
}
void launch_broaden_adj(bool, const HChunk *, int64_t, const CrystalPlan *, bool, const int64_t *, const double *,
                        const int32_t *, const double *, double, double, int64_t, double, double, double2 *,
                        hipStream_t) {
  reached("broaden_adj");
}
void launch_sf_bw(bool, bool, const SfItem *, int64_t, int64_t, const CrystalPlan *, const int64_t *, const int16_t *,
                  const int16_t *, const int16_t *, const double *, const double *, double, const AtomRec *,
                  const SpeciesRun *, const int32_t *, const double *, const CoeffF *, const void *, const double2 *,
                  double *, double *, double *, double *, double *, int, hipStream_t) {
  reached("sf_bw");
}
void launch_atom_bw(bool, bool, const BwItem *, int64_t, const CrystalPlan *, const int64_t *, const int16_t *,
                    const int16_t *, const int16_t *, const double *, const double *, const double *, const AtomRec *,
                    const SpeciesRun *, const int32_t *, const double *, const CoeffF *, int, int, double *,
                    hipStream_t) {
  reached("atom_bw");
}
void launch_march_dollase(const HChunk *, int64_t, const CrystalPlan *, const int64_t *, const int16_t *,
                          const int16_t *, const int16_t *, const double *, const double *, double *, hipStream_t) {
  reached("march_dollase");
}
void launch_noise(int64_t, uint64_t, double, double, double *, hipStream_t) { reached("noise"); }
void launch_broaden_caglioti(bool, const CrystalPlan *, int64_t, const int64_t *, bool, const double *, const int32_t *,
                             const double *, double, double, int64_t, double, double, double, double, double, double *,
                             hipStream_t) {
  reached("caglioti");
}
void launch_bw_finish(const AbItem *, int64_t, bool, const CrystalPlan *, int64_t, const int64_t *, const double *,
                      const double *, const int32_t *, const double *, double *, double *, double *, hipStream_t) {
  reached("bw_finish");
}
}  // namespace xrd
