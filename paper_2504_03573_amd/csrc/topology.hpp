// Host mesh preprocessing (no device code).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "context.hpp"
#include "launch.hpp"
#include "sipdg.h"

namespace sipdg {

struct Topology {
    int dim = 0, nprob = 0;
    int64_t ne = 0, ndof = 0, nfaces = 0;
    int64_t vgeo_len = 0, fgeo_len = 0, tbuf_len = 0;
    int64_t n_interior = 0, n_boundary = 0, n_nonconf = 0, n_trace_points = 0;
    int64_t n_int_trace_points = 0, n_bnd_trace_points = 0;
    int64_t orient_count[8] = {0};
    std::vector<int> order, elem_prob, face_prob;
    std::vector<double> lambda, corners, h, sigma, tau0;
    std::vector<int64_t> xoff, voff, qoff, boff, foff, toff;
    std::vector<int64_t> prob_elem_off, prob_dof_off, prob_face_off;
    std::vector<FaceTopo> faces;
    std::vector<FaceRef> eface;
};

int build_topology(int nprob, const sipdg_mesh_desc *descs, Topology &T, std::string &err);

}  // namespace sipdg
