// Circuit store: an ordered list of levels (the paper's nets, Section III-B),
// each a set of gates on disjoint qubits, with stable ids and an edit record.
#pragma once
#include <cstddef>
#include <cstdint>
#include <unordered_map>
#include <vector>

namespace qtask {

struct Gate {
    uint64_t id = 0;
    uint64_t level = 0;  // level id
    int kind = 0;
    int nq = 0;
    int q[3] = {-1, -1, -1};
    int np = 0;
    double p[3] = {0, 0, 0};
};

struct Level {
    uint64_t id = 0;
    uint64_t version = 0;             // bumped by every gate insert/remove in the level
    uint64_t qmask = 0;               // qubits used by its gates
    std::vector<uint64_t> gates;      // gate ids in insertion order
};

class Circuit {
public:
    explicit Circuit(int n) : n_(n) {}

    int n() const { return n_; }
    size_t num_levels() const { return order_.size(); }
    uint64_t num_gates() const { return gates_.size(); }

    // Each returns a qtask status code; on error nothing changes.
    int insert_level(uint64_t after, uint64_t *out);
    int remove_level(uint64_t level);
    int insert_gate(uint64_t level, int kind, const int32_t *qubits, int nq,
                    const double *params, int np, uint64_t *out);
    int remove_gate(uint64_t gate);
    int level_at(uint64_t index, uint64_t *out) const;

    const Level &level_by_index(size_t i) const { return levels_.at(order_[i]); }
    const Gate &gate(uint64_t id) const { return gates_.at(id); }
    bool has_gate(uint64_t id) const { return gates_.count(id) != 0; }

    // Index of the first level modified since the last clear_edits();
    // SIZE_MAX when nothing changed.  Every level at or after it may differ.
    size_t first_edited() const { return first_edited_; }
    bool edited() const { return first_edited_ != SIZE_MAX; }
    void clear_edits() { first_edited_ = SIZE_MAX; }
    void mark_all_edited() { first_edited_ = 0; }

private:
    long index_of(uint64_t level_id) const;
    void touch(size_t index) {
        if (index < first_edited_) first_edited_ = index;
    }

    int n_;
    std::vector<uint64_t> order_;  // level ids in circuit order
    std::unordered_map<uint64_t, Level> levels_;
    std::unordered_map<uint64_t, Gate> gates_;
    uint64_t next_level_ = 1;
    uint64_t next_gate_ = 1;
    size_t first_edited_ = SIZE_MAX;
};

}  // namespace qtask
