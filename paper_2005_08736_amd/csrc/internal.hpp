// Internal declarations shared by the HIP sources of libhgks (not part of the ABI).
#pragma once

#include "device_common.hpp"

namespace hgks {

void launch_dt(const Geo& g, const double* part, Ctrl* ctrl, double dt_fixed, int hist, hipStream_t st);
template <typename TF>
void launch_stage1(const Geo& g, const double* qn, const TF* fl, double* qs, double* rr, Ctrl* ctrl, int step,
                   hipStream_t st);
template <typename TF>
void launch_stage2(const Geo& g, const double* rr, const TF* fl, const double* qn, double* qout, Ctrl* ctrl,
                   double* part, double* mpart, int step, hipStream_t st);
// constant bulk momentum: the force from the stage-2 block sums in mflux, then
// applied to qout with the CFL block maxima
void launch_bulk_force(const Geo& g, const double* qn, double* qout, Ctrl* ctrl, double* mflux, double m_b,
                       double* part, int step, hipStream_t st);
void launch_check_state(const Geo& g, const double* q, Ctrl* ctrl, double* part, int step, hipStream_t st);
size_t speed_partials(const Geo& g);
void launch_reset_ctrl(Ctrl* ctrl, hipStream_t st);
template <typename TF>
void launch_operator(const Geo& g, const TF* fl, double* L, double* dL, hipStream_t st);
template <typename TF>
void launch_export_flux(const Geo& g, int dir, const TF* fl, double* F, double* dF, hipStream_t st);
// the y-face fluxes of the two wall rows (channel), from the y-direction flux array
template <typename TF>
void launch_export_wall_flux(const Geo& g, const TF* fl, double* F, double* dF, hipStream_t st);
void launch_flux_fused(const Geo& g, int dir, bool stage2, const double* q, double* fl, const int* stop,
                       hipStream_t st);
void launch_flux_fused(const Geo& g, int dir, bool stage2, const double* q, float* fl, const int* stop,
                       hipStream_t st);
void launch_flux_z(const Geo& g, int dir, bool stage2, const double* q, double* fl, const int* stop, const double* dtp,
                   hipStream_t st);
void launch_flux_z(const Geo& g, int dir, bool stage2, const double* q, float* fl, const int* stop, const double* dtp,
                   hipStream_t st);
// mode Z with WENO-Z in characteristic variables
void launch_flux_zc(const Geo& g, int dir, bool stage2, const double* q, double* fl, const int* stop,
                    const double* dtp, hipStream_t st);
void launch_flux_zc(const Geo& g, int dir, bool stage2, const double* q, float* fl, const int* stop,
                    const double* dtp, hipStream_t st);
void launch_operator_vjp(const Geo& g, int dir, bool f32, const double* q, const double* A, const double* B,
                         double cLA, double cLB, double cDA, double cDB, double* G, double* lam, hipStream_t st);
void launch_operator_vjp_z(const Geo& g, int dir, const double* q, const double* A, const double* B, double cLA,
                           double cLB, double cDA, double cDB, const double* dtp, double* lam, hipStream_t st);
void launch_axpby(double a, const double* X, double b, const double* Y, double* out, long long n, hipStream_t st);
void launch_fill(double* out, double v, long long n, hipStream_t st);
void launch_set_dt(Ctrl* ctrl, double dt, hipStream_t st);
void launch_copy(const double* src, double* dst, long long n, hipStream_t st);
void launch_diagnostics(const Geo& g, const double* q, double* part, double* out, hipStream_t st);
size_t diag_partial_doubles();
// histogram of the normalized dilatation, in the diagnostics' partial buffer
constexpr int kPdfMaxBins = 4096;
void launch_dilatation_pdf(const Geo& g, const double* q, double* part, int nbins, double lo, double hi,
                           hipStream_t st);
size_t dilatation_pdf_rms_offset();
size_t dilatation_pdf_counts_offset();
// theta / theta_rms on one plane of cells, written to out (device)
void launch_dilatation_slice(const Geo& g, const double* q, double* part, int axis, int index, double* out,
                             hipStream_t st);
// plane-averaged profiles per y row: kNProfile doubles per row
constexpr int kNProfile = 11;
void launch_plane_profiles(const Geo& g, const double* q, double* out, hipStream_t st);

}  // namespace hgks
