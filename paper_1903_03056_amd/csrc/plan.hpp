// Internal plan object of the collision library and the device launch interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "dgfs.h"

namespace dgfs {

// Launch geometry of the fused gain kernel for one velocity resolution N:
// CH   chunks of the output grid along x (each work item owns x-indices = c mod CH),
// CZ   thread groups sharing each y/z pencil of the chunk (group g keeps the outputs
//      with index = g mod CZ); CZ = 0: the shifted fields are formed on the matrix cores
//      (gain_mfma.hip).
struct GainGeometry {
    int CH;
    int CZ;
};

// The default: the first compiled geometry, skipping the matrix-core ones (CZ = 0: FP32
// VHS plans of the circular form) unless matrix_ok.
bool gain_geometry(int N, int precision, GainGeometry* g, bool matrix_ok = true);
// Bytes per (node, species) of the matrix-core gain's prepared input (N = 32): f split into
// FP16 hi and lo, the alternating x-sum plane split likewise, and 64 FP32 scalars.
constexpr size_t mfma_prep_bytes = (2 * 32768 + 2048) * 2 + 64 * 4;
int tile_candidates(int N, int precision, GainGeometry* out, int max);  // compiled geometries

// One "gain class": the S_q field sum_p w A_p B_p with A = f^i shifted by +a rho sigma_p,
// B = f^j shifted by -b rho sigma_p.  With an antipodal design one class serves both
// orderings of an unlike pair, and a like pair needs only half of the directions.
//
// With a VSS kernel the kernel mode depends on sigma, so the directions are not summed:
// a class holds one direction, whose complex product S is transformed whole, and the
// sphere weight goes into the kernel-mode tables.
struct GainClass {
    int i, j;
    double a, b;
    int ndir;        // directions of this class
    int dir_offset;  // first global direction index in the phase tables
    double weight;   // sphere weight per direction (4 pi / M, doubled for a halved like pair; 1 for VSS)
    std::vector<int> dirs;  // design point of each direction
};

struct PairParams {
    double a, b, gamma, C, R, alpha;
    std::vector<double> rho, wrho;
};

// Device-side integer descriptors (all int32):
//   class:  i, j, ndir, dir_offset
//   slot:   species, gain_begin, gain_count, loss_begin, loss_count
//   gain term: class, F table
//   loss term: species j, G table
struct SlotSet {
    int nslots = 0;
    std::vector<int> slots, gterms, lterms;
    std::vector<int> cuses;  // per class: (slot, F table) of its first and second use, -1 if none
    size_t off_slots = 0, off_gterms = 0, off_lterms = 0, off_cuses = 0;  // byte offsets in the device block
};

}  // namespace dgfs

struct dgfs_plan {
    int s = 0, N = 0, M = 0, nrho = 0, precision = 0;
    double L = 0;               // box half-width (the widest box with species-specific grids)
    std::vector<double> mass;
    std::vector<double> Ls;     // [s] half-width of each species' grid
    std::vector<unsigned char> mask;  // [s*s] ordered pairs evaluated by this plan
    dgfs::GainGeometry geo{};
    std::vector<double> sigma;  // design, [M][3]
    bool antipodal = false;
    bool vss = false;           // some pair has alpha > 1: sigma-dependent kernel-mode tables
    std::vector<dgfs::PairParams> pair;  // [s*s]
    std::vector<dgfs::GainClass> classes;
    int total_dirs = 0;
    int nftab = 0, ngtab = 0, K2 = 0;
    dgfs::SlotSet sum_slots, pair_slots;

    int device = 0;
    void* dev = nullptr;  // one block holding every table
    size_t dev_bytes = 0;
    // byte offsets of the tables in `dev`
    size_t off_kx = 0, off_yz = 0, off_nyq = 0, off_F = 0, off_G = 0, off_tw = 0, off_cls = 0, off_wdir = 0;
    // matrix-core gain (geometry CZ = 0): split-FP16 shift-matrix operands and Nyquist
    // coefficients per (direction, rho, field)
    size_t off_mtab = 0, off_msc = 0;
    size_t off_minv = 0;  // (s+4)^2 doubles, inverse Gram matrix of the invariants
    // plain per-point FP64 path (FP64 plans only): phases [s*s][nrho][M][2][3][N], F [s*s][nrho][K2]
    size_t off_plain_ph = 0, off_plain_F = 0;

    // Species-specific grids: one single-grid sub-plan per distinct pair box L_ij, each
    // evaluating the ordered pairs whose wider box it is.  Empty for a single-grid plan.
    struct GridPart {
        dgfs_plan* plan = nullptr;
        double L = 0;
        std::vector<int> species;         // global index of each local species
        std::vector<long long> t_in;      // byte offset in `dev` of the map own grid -> L, or -1
        std::vector<long long> t_out;     // byte offset in `dev` of the map L -> own grid, or -1
    };
    std::vector<GridPart> parts;

    // Dealiased form (linear convolution): the companion plan on the 3N/2 grid whose
    // tables the padded gain and loss use; this plan keeps the conservation tables.
    dgfs_plan* inner = nullptr;

    size_t elem() const { return precision == DGFS_FP64 ? sizeof(double) : sizeof(float); }
    size_t n3() const { return size_t(N) * N * N; }
    // workspace bytes per node, and the alignment slack added once per call
    size_t ws_per_node(bool pairs) const;
    size_t ws_slack() const { return parts.empty() ? 4 * 256 : 12 * 256; }
};

namespace dgfs {
// Launch the full collide pipeline for nb nodes on `stream`.
// ev: NULL, or 6 events recorded at the stage boundaries of the slice.
hipError_t launch_collide(const dgfs_plan& p, const void* f, void* Q, int64_t nb, void* ws,
                          bool pairs, hipStream_t stream, hipEvent_t* ev);
// The dealiased pipeline (vss_24.hip: N = 16, dealias_36.hip: N = 24, vss_48.hip: N = 32,
// dealias_72.hip: N = 48).
hipError_t run_dealias_16(const dgfs_plan& outer, const dgfs_plan& inner, const void* f, void* Q, int nb, void* ws,
                          bool pairs, hipStream_t st, hipEvent_t* ev);
hipError_t run_dealias_24(const dgfs_plan& outer, const dgfs_plan& inner, const void* f, void* Q, int nb, void* ws,
                          bool pairs, hipStream_t st, hipEvent_t* ev);
hipError_t run_dealias_32(const dgfs_plan& outer, const dgfs_plan& inner, const void* f, void* Q, int nb, void* ws,
                          bool pairs, hipStream_t st, hipEvent_t* ev);
hipError_t run_dealias_48(const dgfs_plan& outer, const dgfs_plan& inner, const void* f, void* Q, int nb, void* ws,
                          bool pairs, hipStream_t st, hipEvent_t* ev);
// out != NULL: out = projection of Q (FP64); fstate != NULL: fstate += dt * projection.
hipError_t launch_conserve(const dgfs_plan& p, const void* Q, double* out, void* fstate, double dt, int64_t nb,
                           hipStream_t stream);
// Copy (Tm == NULL) or interpolate (Tm = [N][N] one-dimensional map, applied along each
// axis) nb fields of N^3 values with per-node strides (in elements), storing or adding.
// tmp: 2 nb N^3 values of scratch.
hipError_t launch_move(const dgfs_plan& p, const void* in, int64_t in_stride, void* out, int64_t out_stride,
                       const void* Tm, int64_t nb, bool accumulate, void* tmp, hipStream_t stream);
// out = a x + b y over n values of the plan precision.
hipError_t launch_axpby(const dgfs_plan& p, const void* x, const void* y, void* out, double a, double b, int64_t n,
                        hipStream_t stream);
// Workspace bytes per node of the dealiased pipeline on an N-grid plan (NI = 3N/2):
// f_hat on N, the padded f_hat and the complex interpolant on NI, the class partials on
// NI, the loss spectra on NI and the kept modes on N.
inline size_t dealias_ws_per_node(size_t elem, int N, int s, int ncls, int nrho, int nslots) {
    const size_t c = 2 * elem, N3 = size_t(N) * N * N, NI = size_t(3 * N / 2), NI3 = NI * NI * NI;
    return c * (size_t(s) * N3 + 2 * size_t(s) * NI3 + size_t(ncls) * nrho * NI3 + size_t(nslots) * NI3 +
                size_t(nslots) * N3) + 7 * 256;
}
// dgfs_collide with the caller's workspace (api.cpp): the batch runs in slices of as many
// nodes as ws_bytes holds.
dgfs_status collide_with_workspace(const dgfs_plan* plan, const void* f, void* Q, int64_t batch, void* ws,
                                   size_t ws_bytes, void* stream);
// Record the error text returned by dgfs_last_error and return st (api.cpp).
dgfs_status set_error(dgfs_status st, const std::string& msg);
// Plain per-point FP64 path (plain.hip).
size_t plain_ws_bytes(const dgfs_plan& p);
hipError_t launch_collide_plain(const dgfs_plan& p, const double* f, double* Q, int64_t nb, void* ws,
                                hipStream_t stream);
}  // namespace dgfs
