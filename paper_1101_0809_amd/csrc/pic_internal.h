// pic_internal.h -- internal declarations of the gfx950 PIC library: the
// context, the particle-buffer layouts and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/pic.h"

namespace pic {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxSpecies = 4;
constexpr size_t kAlign = 256;  // alignment of every carved buffer
constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, each with its own L2

// Tile edge (cells) of the particle-step kernel, per dimensionality.
constexpr int kTile3 = 8;
constexpr int kTile2 = 16;

// 3D particle kernel LDS layout, per precision.  A particle inside a tile's
// region may sit up to MX cells outside the tile along x and M cells along y
// and z.  The field tile (E^n, B^n) covers LFX x LFY x LFY cells, with rows of
// FROW values and planes of FPLANE; the FP64 current tile covers LJX x LJY x
// LJY cells, with rows of JROW and planes of JPLANE doubles.  The strides agree
// modulo 32, so the field base index and the current base index of a cell have
// the same residue: the cell's lane class, shared by the sort (which places
// particles by class) and the kernel.  FP32 mode stores its field tile in
// FP32, which leaves room for a margin of 3 along x: fewer particles leave
// their tile's region between sorts when they drift along x.  Its rows of 18
// and planes of 216 and 280 spread a tile's cells evenly over the 32 lane
// classes and keep a gather stencil within one LDS base register's reach.
template <class R>
struct Tile3;
template <>
struct Tile3<double> {
    static constexpr int MX = 1, M = 1;
    static constexpr int FROW = 14, FPLANE = 168, JROW = 14, JPLANE = 200;
};
template <>
struct Tile3<float> {
    static constexpr int MX = 3, M = 1;
    static constexpr int FROW = 18, FPLANE = 216, JROW = 18, JPLANE = 280;
};
template <class R>
struct Tile3Dims : Tile3<R> {
    using L = Tile3<R>;
    static constexpr int LFX = kTile3 + 2 + 2 * L::MX, LFY = kTile3 + 2 + 2 * L::M;
    static constexpr int LJX = kTile3 + 4 + 2 * L::MX, LJY = kTile3 + 4 + 2 * L::M;
    static constexpr int NJ = LJY * L::JPLANE;  // doubles per current component
    static_assert(L::FROW >= LFX && L::FPLANE >= LFY * L::FROW, "field rows and planes hold the region");
    static_assert(L::JROW >= LJX && L::JPLANE >= LJY * L::JROW, "current rows and planes hold the region");
    static_assert((L::JROW - L::FROW) % 32 == 0 && (L::JPLANE - L::FPLANE) % 32 == 0,
                  "field and current strides agree mod 32");
    static_assert(kTile3 - 1 + 2 * L::MX < 16 && kTile3 - 1 + 2 * L::M < 16, "region offsets fit 4 bits");
};

// Lane classes: LDS serves 128 bytes per clock, 16 lanes of 8-byte values (FP64
// fields and the current tile) or 32 lanes of 4-byte values (FP32 fields).
template <class R>
constexpr int lane_classes() { return sizeof(R) == 8 ? 16 : 32; }

// Class of a cell at offset rel from its tile's first cell (rel inside the
// tile region): its field-tile base index modulo the lane classes.
template <class R>
__host__ __device__ inline int cell_class3(int rx, int ry, int rz)
{
    using L = Tile3<R>;
    return ((rx + 1 + L::MX) + (ry + 1 + L::M) * L::FROW + (rz + 1 + L::M) * L::FPLANE) & (lane_classes<R>() - 1);
}

// Particle arrays of one copy (the library keeps two for out-of-place sorts).
// FP64 mode: pos[a] are double absolute positions in [0, N_a).
// FP32 mode: cell packs (i | j << 11 | k << 22), pos[a] are float offsets in [0, 1).
struct PartArrays {
    void* pos[3];
    void* mom[3];
    void* weight;
    uint32_t* cell;  // FP32 mode only
    int64_t* id;
};

struct Species {
    pic_species_desc d{};
    int64_t n = 0;
    char* buf = nullptr;
    size_t bytes = 0;
    PartArrays cur{}, alt{};
    uint32_t* key = nullptr;   // sort key per particle
    uint32_t* rank = nullptr;  // rank within the key bucket (from the histogram atomics)
    uint32_t* dest = nullptr;  // final slot of each cell-sorted position (sort scratch)
    uint32_t* src = nullptr;   // particle that moves to each final slot (sort scratch)
    int64_t* tile_start = nullptr;  // ntiles + 1 entries
    bool sorted = false;
    int swapped = 0;           // 1: cur is the buffer's second copy
};

// Grid constants handed to kernels by value.
struct GridK {
    int n[3];        // cells per axis
    int nt[3];       // tiles per axis
    int tile[3];     // tile edge per axis (1 for z in 2D)
    int dims;
    int ntiles;
    int64_t ncell;
    double cfl[3];   // c dt / d_a
    double half_cfl[3];
    double dt, c;
    double bext[3];
    double inv_vol;  // 1 / (dx dy dz)
    double jscale[3];  // -(1/4) d_a / dt / V : xi -> J factor per unit charge
    double fourpidt;   // 4 pi dt
    double inv_h[3];   // 1 / d_a
    // plane-wave source (see pic_grid_desc): kind, plane, amplitude, omega, ramp
    int src_kind;
    int src_plane;
    double src_amp, src_omega, src_ramp;
    double* aux;       // auxiliary line: E^y[PIC_AUX] then B^z[PIC_AUX] (workspace)
    int field_form;    // 0: B carried; 1: vector potential carried (B = curl A)
};

struct Ctx {
    pic_grid_desc g{};
    GridK k{};
    double* fields = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    // workspace carve-up
    double* rho_bg = nullptr;   // immobile charge density
    double* r0 = nullptr;       // Gauss reference R^0
    double* rho_m = nullptr;    // scratch: mobile charge density
    uint32_t* hist = nullptr;   // nkeys + 1 counts / offsets
    uint32_t* scan_part = nullptr;
    double* red = nullptr;      // reduction partials
    double* bn = nullptr;       // B^n of the current step (3 planes), read by the particles
    double* adj = nullptr;      // adjoint scratch (3 planes): lambda_J of a reverse step
    double* avec = nullptr;     // vector potential A^{n-1/2} (3 planes, field form 1 only)
    unsigned long long* counters = nullptr;  // [0] range errors, [1] fallback particles,
                                             // [2] particles processed, [3] migrants
    unsigned int* mig_n = nullptr;  // per-tile migrant bucket counters (3D particle step)
    uint32_t nkeys = 0;
    Species sp[kMaxSpecies];
    int nsp = 0;
    int64_t step = 0;
    int since_sort = 0;
    bool r0_valid = false;
    std::string err;
};

size_t align_up(size_t v, size_t a);

// ---- launchers (stream = hipStream_t) ----
hipError_t launch_field_half_b(const Ctx& c, hipStream_t s);
// Both B half steps of a step; also zeroes zero[0 .. nzero) first (counters).
hipError_t launch_field_half_b_pair(const Ctx& c, hipStream_t s, unsigned long long* zero = nullptr,
                                    int nzero = 0);
hipError_t launch_field_update_e(const Ctx& c, hipStream_t s, int64_t step);
// Field form 1: A^{n+1/2} = A^{n-1/2} - c dt E^n, B^n = curl_h A^n into bn,
// B^{n+1/2} = curl_h A^{n+1/2} into the B planes (zeroing counters as above).
hipError_t launch_field_half_a_pair(const Ctx& c, hipStream_t s, unsigned long long* zero = nullptr, int nzero = 0);
// B planes = curl_h A (field form 1).
hipError_t launch_b_of_a(const Ctx& c, hipStream_t s);
hipError_t launch_particle_step(Ctx& c, Species& sp, hipStream_t s);
hipError_t launch_load(Ctx& c, Species& sp, int64_t n, const double* x, const double* w,
                       const double* weight, hipStream_t s);
hipError_t launch_get(const Ctx& c, const Species& sp, double* x, double* w, double* weight,
                      int64_t* id, hipStream_t s);
hipError_t launch_deposit_only(const Ctx& c, const double* x0, const double* x1,
                               const double* charge, int64_t n, double* J, hipStream_t s);
hipError_t launch_rho(const Ctx& c, const Species& sp, double* rho, hipStream_t s);
hipError_t launch_rho_raw(const Ctx& c, const double* x, const double* weight, double charge,
                          int64_t n, double* rho, hipStream_t s);
hipError_t launch_sort(Ctx& c, Species& sp, hipStream_t s);
// Alternating order 2 1/2 (grid order 2, FP64): the particle step, the
// current of given moves and the charge density of positions x[ax][p].
hipError_t launch_particle_step_o2(Ctx& c, Species& sp, hipStream_t s);
hipError_t launch_deposit_only_o2(const Ctx& c, const double* x0, const double* x1, const double* charge,
                                  int64_t n, double* J, hipStream_t s);
hipError_t launch_rho_o2(const Ctx& c, const double* const x[3], const double* weight, int64_t n, double q,
                         double* rho, hipStream_t s);
// The conventional interpolation of Eq. wrong1 (grid interp 1, order 1, FP64).
hipError_t launch_particle_step_conv(Ctx& c, Species& sp, hipStream_t s);
// rho_m (N doubles) and part (diag_partials_doubles) are scratch; null: the workspace's.
hipError_t launch_diag(Ctx& c, pic_diag* out, hipStream_t s, double* rho_m = nullptr, double* part = nullptr);
hipError_t launch_capture_r0(Ctx& c, hipStream_t s, double* rho_m = nullptr);
size_t diag_partials_doubles(int nsp);
// The static scratch of pic_diagnostics_static: its size, the doubles a
// context needs of it, and its device address on the current device.
constexpr size_t kStaticScratchBytes = (size_t)20 << 20;
size_t static_scratch_doubles(const Ctx& c);
hipError_t static_scratch_address(double** out);
// rho of the mobile species (into the workspace's rho_m) plus the background, into out.
hipError_t launch_total_rho(Ctx& c, double* out, hipStream_t s);
// Electrostatic field of the charge density rho (Eqs. poiphi, egradphidis)
// into E; with neutralize, minus the mean of rho is first added to the
// background.  Conjugate gradients to a relative residual tol; synchronizes.
hipError_t solve_poisson(Ctx& c, double* rho, bool neutralize, double tol, int64_t max_iter, int64_t* iters,
                         double* rel_residual, hipStream_t s);
hipError_t launch_adjoint_seed(const Ctx& c, double* lam, hipStream_t s);
// record == nullptr: the state before the step is the context's own; else a
// record written by launch_adjoint_record.
// by_id: particle adjoints indexed by id; else by storage position (of the
// record, or of the context).
hipError_t launch_adjoint_step(const Ctx& c, const void* record, bool by_id, double* lam, double* const* lam_x,
                               double* const* lam_w, double* lam_bext, hipStream_t s);
// Particle adjoints from the storage order of record `from` to that of `to`
// (null: id order); uses the species' sort-key scratch.
hipError_t launch_adjoint_reorder(Ctx& c, const void* from, const void* to, const double* const* in_x,
                                  const double* const* in_w, double* const* out_x, double* const* out_w,
                                  hipStream_t s);
size_t adjoint_record_bytes(const Ctx& c);
hipError_t launch_adjoint_record(const Ctx& c, void* record, hipStream_t s);

}  // namespace pic
