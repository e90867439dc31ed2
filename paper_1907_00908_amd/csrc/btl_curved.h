// Host-side term lists of the general membrane condition for membranes at an
// angle to the lattice links (Sec. 2.4.2 and Appendix B).  Internal to
// libbtlbm.
#pragma once

#include <stdint.h>

#include <vector>

#include "btl_internal.h"
#include "btlbm.h"

namespace btl {

// The membrane links of one geometry that carry a membrane normal, kept from
// btl_create: everything their term lists need besides the permeabilities,
// the time step and the lattice.
struct CurvedGeom {
    int32_t n[3];
    int32_t bc[3];
    std::vector<uint32_t> comp;    // compartment of every site
    std::vector<uint8_t> phase;    // phase of every compartment
    struct Link {
        int64_t s;      // receiving site
        int32_t d;      // pull direction (1..6: +x, -x, +y, -y, +z, -z)
        double dist;    // distance from the site to the membrane, units of dx
        double nrm[3];  // the membrane normal on the link (either orientation)
    };
    std::vector<Link> links;
    int64_t cv_off = 0;            // offset of the geometry's index table
    int32_t h0 = 0, nh = 0;        // its links in the head table of the last build
};

// Collects the membrane links of g (g.link_normal and g.link_delta set).
// False when the normal of a membrane link is not finite or is zero.
bool curved_collect(const btl_geom& g, CurvedGeom& out);

// Term lists of every link of cg for the lattice nq (7: D3Q7, 5: D2Q5 on a
// single layer), time step dt (ms), spacing dx (um) and permeabilities kappa
// [P*P] (um/ms).  idx ([6][nsites], filled with -1 by the caller) receives
// for each link that takes the condition the index of its entry in heads
// ({first term, number of terms, receiving site's direction-0 element, pull
// direction}); the terms are appended to terms, with population offsets and
// face wraps in the kernel's layout of the lattice.  False when the tables
// would pass 2^31 - 1 entries.
bool curved_terms(const CurvedGeom& cg, int nq, double dt, double dx, const double* kappa,
                  int P, int32_t* idx, std::vector<int4>& heads, std::vector<CvTerm>& terms);

}  // namespace btl
