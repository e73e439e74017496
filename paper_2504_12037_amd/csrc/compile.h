// Host-side instance compiler: validates a tnvan_instance and turns its
// width set and elimination order into the step program of program.h.
// Pure C++ (no HIP), so it is also built and tested on machines without a GPU.
#pragma once
#include <string>
#include <vector>

#include "../../include/tnvan.h"
#include "program.h"

namespace tnvan {

struct HostProgram {
  std::vector<InstDesc> insts;
  std::vector<StepDesc> steps;
  std::vector<InputDesc> inputs;
  std::vector<uint16_t> gtab;     // gather tables of SINGLE steps' inputs
  std::vector<uint32_t> gtab2;    // split gather tables of wide steps' inputs (2 x 1024 each)
  std::vector<double> esmall;     // per EdgeDesc: exp(-2 beta |J|), negated for J < 0
  std::vector<EdgeDesc> edges;
  std::vector<double> T;          // all step tables, FP64
  std::vector<int32_t> fld_ptr;   // per instance: nr + 1 entries (local)
  std::vector<int32_t> fld_w;     // W index of each W-neighbour
  std::vector<double> fld_J;      // its coupling
  std::vector<double> hR;         // h on R positions
  std::vector<int32_t> wr_pos, wr_w, wr_edge;   // W-R edges
  std::vector<double> wr_J;
  std::vector<int32_t> rr_edge;   // R-R edges (global edge id per instance)
  std::vector<double> rr_J;
  std::vector<int32_t> ww_a, ww_b;  // W-W edges as W indices
  std::vector<int32_t> ww_e;        // W-W edges: edge index
  std::vector<double> ww_J;
  std::vector<double> hW;           // h on W indices (for E_1)
  std::vector<int32_t> vr, wv;      // R position -> vertex, W index -> vertex
  std::vector<int32_t> hidden;      // per instance
  std::vector<int32_t> depth;       // per instance: hidden layers (1 when H = 0)
  std::vector<int64_t> flops_fwd;   // per instance, per sample
  std::vector<int32_t> hw_off;      // per instance offset into hW
  std::vector<int32_t> fld_wr;      // W-R edge (local index) of each fld entry
  // transfer-matrix form
  std::vector<ChainInst> cinst;     // per instance
  std::vector<ChainDesc> chains;
  std::vector<ChainStep> csteps;
  std::vector<float> Tp, Tt;        // padded FP32 tables
  std::vector<uint16_t> Tb;         // padded BF16 tables (operand order)
  std::vector<float> Tl;            // per chain: FP32 tables with rows padded by one
  std::vector<uint16_t> Tbl;        // per chain: BF16 operand-order tables
  std::vector<EdgeDesc> cedges;     // per chain: the edges of its steps
  std::vector<float> Tr, Tq;        // register-resident operand tables
  std::vector<uint16_t> Trb;
  std::vector<uint16_t> Ts3;        // per chain step: split-BF16 operand tables
  std::vector<int32_t> xcol;        // 16 adjoint column codes per chain step
  std::vector<float> Tsx;           // per chain step: S_x and S_o operand tables
  std::vector<int32_t> Tdq;         // per chain step: adjoint destinations [lane][4]
  // adjoint output maps: vertex -> R position (-1 on W), edge -> partial
  // column (-1 on W-W edges), and the dbeta coefficient of every column
  std::vector<int32_t> col_out;      // per partial column: its adjoint output (vertex, or n + edge)
  std::vector<double> pcoef_out;     // per adjoint output: dbeta coefficient of its column, or 0
  std::vector<int32_t> cf_w, cf_r;  // 4 W-neighbour slots per R position (index, W-R edge)
  std::vector<float> cf_J;          // their couplings
};

// Appends one instance to P.  Returns TNVAN_OK or an error code with msg.
tnvan_status compile_instance(const tnvan_instance &in, int max_width,
                              HostProgram &P, std::string &msg);

}  // namespace tnvan
