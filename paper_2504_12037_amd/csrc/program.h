// Compiled contraction program of one or more disorder instances.
//
// The conditional partition function of the remainder R (Sec. 2, Eqs. 3-4)
// is contracted by eliminating R group by group along the given order.  A
// step eliminates a group G of consecutive order positions and produces a
// message over the scope S_out (the not-yet-eliminated R vertices it still
// touches).  Per sample s_W the step computes
//
//   out[o] = sum_x T[x, o] * d[x] * prod_k m_k[idx_k(o, x)]
//
// where x runs over the 2^g states of G, o over the 2^w states of S_out,
// T is the static product of the Boltzmann matrices (Eq. 2) of the R-R
// edges the step consumes (normalised so that every factor is <= 1), d is
// the product of the per-sample unary factors of G (the W-R couplings act on
// R as fields, the "extra interaction" of Sec. 2) and m_k are the messages of
// earlier steps whose scope meets G.
//
// Bit conventions: a message entry index has bit b set when the b-th vertex
// of its scope has spin -1; the combined step index is (x << w) | o.
//
// This header is shared by the host compiler and the device kernels only.
#pragma once
#include <stdint.h>

namespace tnvan {

enum StepKind : int32_t {
  // at most one input message and its scope is exactly G (same bit order);
  // out = A . T with A[x] = d[x] m[x]: a dense batched product
  STEP_DENSE = 0,
  // g == 1 with any inputs: gather-product per output entry
  STEP_SINGLE = 1,
};

constexpr int kMaxScope = 24;   // bits of any message / input scope
constexpr int kMaxW = 20;       // output scope bits
constexpr int kTabW = 14;       // widest step with a full transfer table and gather tables
constexpr int kMaxG = 8;        // group size
constexpr int kMaxInputs = 24;
constexpr int kWideIn = 8;      // most inputs of a wide step
constexpr int kWideEdges = 8;   // most R-R edges a wide step consumes

// Wide steps (single-spin steps with an output scope of kTabW + 1 .. kMaxW
// bits): no 2^(w+1)-entry transfer table (t_off = -1); T[x, o] is formed on
// the fly from the step's edges as the product over them of 1 where
// J s_x s_o > 0, else exp(-2 beta |J|) (esmall holds that value per edge,
// negated for J < 0); each input gathers through two 1024-entry tables
// (gtab2: the entry for the low 10 and for the high 10 bits of o, or-ed).

struct StepDesc {
  int32_t kind;
  int32_t g;          // group size
  int32_t gpos;       // first order position of the group
  int32_t w;          // output scope size (0: the step closes a component)
  int32_t n_in;       // number of input messages
  int32_t in_off;     // index of the first InputDesc
  int64_t t_off;      // offset of T (2^(g+w) entries, index (x << w) | o)
  int32_t off_all;    // arena offset of the output (every message kept)
  int32_t off_fwd;    // arena offset of the output (liveness reuse)
  int32_t n_edge;     // R-R edges folded into T
  int32_t edge_off;   // index of the first EdgeDesc
};

struct InputDesc {
  int32_t step;       // producing step (local index within the instance)
  int32_t nbits;      // scope size of the message
  int32_t xbit;       // SINGLE: bit of the eliminated vertex in this scope
  int32_t gb_off;     // SINGLE: offset of its gather table in gtab (gtab2 for a wide step), or -1
  int32_t omask;      // SINGLE: the output bits that are in this scope (OR of 1 << src[b] >= 0)
  int8_t src[kMaxScope];  // scope bit b -> o-bit index, or -1 for x (SINGLE)
};
// Gather table of a SINGLE step's input (gtab[gb_off + o], 2^w entries):
// the entry of the input message that output entry o reads when the
// eliminated spin is +1; with the spin -1 it reads that entry | 1 << xbit.

struct EdgeDesc {
  int32_t rr;         // local index of the edge among the instance's R-R edges
  int32_t bu;         // combined-index bit of one endpoint (x bits at w..)
  int32_t bv;         // combined-index bit of the other endpoint
  int32_t pad;
};

// Per-instance view, everything as offsets into the flat device arrays.
struct InstDesc {
  int32_t n, n_edges, nw, nr;
  int32_t n_steps, step_off;     // StepDesc range
  int32_t fld_off;               // CSR of W-neighbours of R positions
  int32_t fld_nnz_off;           // offset into fld_w / fld_J
  int32_t hr_off;                // h on R positions
  int32_t n_rr, n_wr;            // R-R and W-R edge counts
  int32_t wr_off;                // WR edge tables (position, w index, edge id)
  int32_t rr_off;                // RR edge tables (edge id, J)
  int32_t ww_off, n_ww;          // WW edge tables for E_1
  int32_t arena_all, arena_fwd;  // arena entries per sample
  int32_t scr_fwd, scr_bwd;      // scratch entries per sample
  int32_t max_w;
  int32_t n_partial;             // nr + n_wr + n_rr
  int32_t vr_off;                // R position -> vertex id
  int32_t wv_off;                // W index -> vertex id
  int32_t pbuf;                  // adjoint: per-state edge partial sums
  double beta;
  double log_const;              // sum of beta |J| over R-R edges
};

// ---------------------------------------------------------------------------
// Transfer-matrix form: when every step is dense and the steps form chains
// (each step consumes exactly the message of the previous step of its chain,
// the first one none, the last one closes the chain), a chain is a sequence
// of batched products [samples x K] . [K x N] with a per-sample diagonal in
// between.  Lattice strips eliminated row by row and the two-block SK
// remainder have this form.  The tables are zero-padded to the matrix-core
// tile sizes.
struct ChainStep {
  int32_t step;       // local step index
  int32_t g, w, gpos;
  int32_t kp;         // padded K for FP32 16x16x4 products (>= 16)
  int32_t kb;         // padded K for BF16 16x16x32 products (>= 32)
  int32_t np;         // padded N (>= 16), or 1 when the step closes the chain
  int32_t n_edge, edge_off;
  int32_t tl_off;     // FP32 [kp][np + 1] table inside the chain's staged block
  int32_t tbl_off;    // BF16 operand-order table inside the chain's staged block
  int32_t ce_off;     // first edge inside the chain's edge list
  int64_t tp_off;     // FP32 [kp][np]
  int64_t tt_off;     // FP32 [np][kp] (transposed, for the adjoint)
  int64_t tb_off;     // BF16 packed in the 16x16x32 operand order
  // register-resident form (see the comment below)
  // (every step of a chain padded with zeros to the chain's rt x rt tiles)
  int64_t tr_off;     // FP32 [nt][xt][lane][4]: T[16xt + 4(lane>>4) + r][16nt + (lane&15)]
  int64_t tq_off;     // FP32 [xt][nt][lane][4]: T[16xt + (lane&15)][16nt + 4(lane>>4) + r]
  int64_t trb_off;    // BF16 [nt][c][lane][8]: T[16(2c + i/4) + 4(lane>>4) + i%4][16nt + (lane&15)]
  int32_t nt16;       // output tiles of 16 (1 for the closing step)
  int32_t xc_off;     // 16 column codes of the adjoint's spin-product matrix
  int64_t sx_off;     // FP32 [xt][lane][4] S_x operands, then [ot][lane][4] S_o operands
  // W-R couplings of the group (at most 4): group spin j and W index in
  // wri = j | (w << 8), the W-R edge in wre
  int32_t n_wri;
  int32_t wri[4];
  int32_t wre[4];
  int32_t dq_off;     // adjoint destinations [lane][4] (see below)
  // split-BF16 operand tables (16x16x32 order, KC = ceil(rt / 2) chunks of 32
  // states; state of element j of lane l in chunk c: 16 (2c + j/4) +
  // 4 (l >> 4) + j % 4, zero past the chain's tiles), BF16 [part][...]:
  //   0/1 forward hi/lo [nt][c][lane][8]: T[state][16 nt + (l & 15)]
  //   2/3 Lambda hi/lo  [xt][c][lane][8]: T[16 xt + (l & 15)][state]
  //   4   S_x           [c][lane][8]:     S_x[state][column l & 15]
  //   5   S_o           [c][lane][8]:     S_o[state][row l & 15]
  // (hi = T rounded to BF16, lo = the rest rounded to BF16)
  int64_t s3_off;
};

// Register-resident layout ("R-layout") of a per-sample vector over 16*KT
// states on one 64-lane wave: lane l holds, for sample l & 15, the states
// 16 t + 4 (l >> 4) + r in register [t][r].  This is the output layout of a
// 16x16x4 FP32 matrix-core product D = T^T A^T (rows = states, columns =
// samples), and the operand layout the next such product reads, so a chain
// runs from register to register; the tables above are the transfer
// matrices permuted into that operand order.
//
// Adjoint column codes (xc): column c of S_x is the spin product
// sigma_u(x) sigma_v(x) with u = code & 0xff, v = (code >> 8) & 0xff
// (v = 31 means a single spin), or a zero column when code < 0.  Columns
// 0..g-1 are the group's spins, then one column per edge with both ends in
// the group.  Every edge of the step stores in EdgeDesc::pad the cell
// (column * 16 + output-spin row) of S_x^T G S_o that holds its correlation
// (row w = the all-ones column of S_o).  The adjoint's 16x16 product
// S_x^T G S_o ends in the R-layout: lane l holds cell (l & 15) * 16 +
// 4 (l >> 4) + r in register r.  dq_off indexes, per lane and register, the
// partial-row column that cell is stored to (-1: none): group spin j's
// magnetisation at cell j * 16 + w, an edge's correlation at its pad.

struct ChainDesc {
  int32_t n_steps, cs_off;   // ChainStep range
  int32_t pos_lo, pos_hi;    // R positions the chain eliminates
  // data a workgroup stages into LDS once for all its waves
  int32_t tl_size;           // floats of the padded FP32 tables of every step
  int32_t tbl_size;          // BF16 entries of the operand-order tables
  int64_t tl_src;            // offset of that block in the FP32 block array
  int64_t tbl_src;           // offset in the BF16 block array
  int32_t e_src, n_e;        // the chain's edges in the chain edge array
  int32_t f_lo, f_hi;        // W-neighbour entries of the chain's positions
  int32_t rt;                // register-resident form: tiles of every step (1, 2, 4, ...)
  int32_t pad;
};

struct ChainInst {
  int32_t ok;                // instance runs in transfer-matrix form
  int32_t n_chains, chain_off;
  int32_t kbuf;              // widest padded K or N of any step
  int32_t npos_max;          // most positions of one chain
  int32_t max_steps;         // longest chain
  int32_t gmax;              // largest group
  int32_t pmax;              // largest per-state edge partial table (kp * (w+1))
  int32_t nw;                // width-set size (spins staged per sample)
  int32_t tl_max;            // largest tl_size of the instance's chains
  int32_t tbl_max;           // largest tbl_size
  int32_t ne_max;            // most edges of one chain
  int32_t nf_max;            // most W-neighbour entries of one chain
  int32_t rtiles;            // widest step in 16-state tiles (register-resident form)
  int32_t rq_ok;             // every step fits the 16-column adjoint products and
                             // every R position has at most 4 W-neighbours
  int32_t pad;
};

}  // namespace tnvan
