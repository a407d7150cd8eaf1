// Work split of the persistent launches, shared by the kernels and by the
// host-side schedule check.
//
// The spectra of one launch form a sequence: sub-array by sub-array, then
// virtual channel v (channel c = v / KS, column part v % KS), then time t.  A
// spectrum of sub-array s costs w_s units (1 for a single sub-array); the
// spectrum k of sub-array s sits at cost offset base_s + k w_s, and workgroup
// g owns the spectra whose offset lies in [g Lc, (g + 1) Lc), Lc = ceil(total
// cost / workgroups).  A workgroup's spectra of one virtual channel are
// contiguous in time and are summed into one partial-accumulator slot of that
// channel; the slots are added in a fixed order at readout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epic {

// ceil(a / b) for b > 0 and any sign of a
__host__ __device__ inline int64_t ceil_div_any(int64_t a, int64_t b) {
    return a <= 0 ? -((-a) / b) : (a + b - 1) / b;
}

// Spectra [k0, k1) of a sub-array of `items` spectra at offsets base + k w
// owned by workgroup g (empty when k0 >= k1).
__host__ __device__ inline void owned_range(int g, int64_t Lc, int64_t base, int64_t w, int64_t items, int64_t* k0,
                                            int64_t* k1) {
    const int64_t c0 = (int64_t)g * Lc;
    int64_t a = ceil_div_any(c0 - base, w), b = ceil_div_any(c0 + Lc - base, w);
    a = a < 0 ? 0 : (a > items ? items : a);
    b = b < 0 ? 0 : (b > items ? items : b);
    *k0 = a;
    *k1 = b;
}

// Slot of workgroup g's piece of virtual channel v, a piece that starts at
// spectrum t of the channel.  When a spectrum costs less than a share
// (w < Lc) consecutive spectra have the same or consecutive owners, so a
// channel's owners are consecutive workgroups and the slot is g's distance
// from the first of them; otherwise every spectrum has an owner of its own
// and the slot is t.  Either way the slot is below min(T, ceil(G / V) + 1)
// for a sub-array of V virtual channels in a launch of G workgroups (its
// spectra cost at most its share of the total, so one channel spans at most
// G / V shares).
__host__ __device__ inline int slot_of(int g, int64_t v, int64_t t, int64_t T, int64_t base, int64_t w, int64_t Lc) {
    if (w >= Lc) return (int)t;
    return g - (int)((base + v * T * w) / Lc);
}

// Column-part-major split of a one-sub-array launch whose image columns are
// split over KS workgroups per spectrum: workgroup g works on column part
// g % KS, and the G / KS workgroups of each part split that part's C x T
// (channel, spectrum) sequence in contiguous runs.  The KS parts of a channel
// then run at the same time on neighbouring workgroups (the same XCD), which
// share the channel's gather program in L2.  G must be a multiple of KS.
struct PartSplit {
    int kpart;   // column part of workgroup g
    int gp;      // its index among the workgroups of that part
    int Gp;      // workgroups per part
};
__host__ __device__ inline PartSplit part_split(int g, int G, int KS) { return PartSplit{g % KS, g / KS, G / KS}; }

}  // namespace epic
