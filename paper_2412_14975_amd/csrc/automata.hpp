// Host-side construction of the automata used by the recognizer.
//
// Pipeline (all on the host, once per expression):
//   regular expression --parse--> syntax tree
//   --position automaton (McNaughton-Yamada, Sect. 4.1)--> NFA N, trimmed
//   --byte classes--> N over K classes
//   --RI-DFA construction (Sect. 3.1)--> B
//   --Nerode partition of B, downgrading with delegation (Sect. 3.4)-->
//   quotient NFA N' (one state per surviving interface state)
//   --RI-DFA construction--> B'      (the chunk automaton of RI_ALGO_RID)
//   --Nerode partition of B'--> minimal DFA (chunk automaton of RI_ALGO_DFA)
//   --powerset construction of N--> RI_ALGO_SUBSET chunk automaton
#pragma once

#include <bitset>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace ri {

struct BuildError : std::runtime_error {
    int code;
    BuildError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

using ByteSet = std::bitset<256>;

// Position NFA: state 0 is q0, states 1..m are symbol occurrences.
struct PositionNfa {
    uint32_t n = 0;
    std::vector<ByteSet> sym;                  // sym[p]: bytes that enter p (p >= 1)
    std::vector<std::vector<uint32_t>> next;   // next[0] = first, next[p] = follow(p)
    std::vector<uint8_t> final;
};

// NFA whose moves are labelled by sets of byte classes.
struct ClassNfa {
    uint32_t n = 0;
    uint32_t K = 0;
    uint32_t mask_words = 0;                   // words of one class mask
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> edges;  // (target, mask id)
    std::vector<uint64_t> masks;               // mask id * mask_words
    std::vector<uint8_t> final;
};

// Deterministic transition graph over K classes; content[p] is the set of
// NFA states that p stands for (sorted), initial[q] the id of {q}.
struct DetAutomaton {
    uint32_t n = 0;
    uint32_t K = 0;
    std::vector<int32_t> delta;                // n*K, -1 = no move
    std::vector<uint8_t> final;
    std::vector<std::vector<uint32_t>> content;
    std::vector<uint32_t> initial;
};

struct Automata {
    // byte classes
    uint32_t K = 0;
    uint8_t cls[256] = {};
    bool empty_language = false;
    bool accepts_empty = false;

    uint32_t nfa_states = 0;         // |Q_N|
    uint32_t ridfa_full_states = 0;  // |P| of B
    PositionNfa pos;                 // trimmed N
    std::vector<uint32_t> cid;       // N state -> N' state
    ClassNfa nq;                     // N'
    DetAutomaton Bq;                 // B'
    std::vector<int32_t> final_id;   // B' state -> minimal DFA id (-1 if not reachable from {0})

    // minimal DFA, canonical numbering, trimmed
    uint32_t dmin_n = 0;
    std::vector<int32_t> dmin_delta;  // dmin_n*K
    std::vector<uint8_t> dmin_final;

    // powerset DFA of N
    uint32_t dsub_n = 0;
    std::vector<int32_t> dsub_delta;
    std::vector<int32_t> dsub_final_id;   // minimal DFA id of each state
    std::vector<uint8_t> dsub_accept;
    std::vector<std::vector<uint32_t>> dsub_content;   // the set of N's states of each state (sorted)

    // N as a chunk automaton over sets of states (the NFA device of Sect. 2),
    // when it has at most kNfaMaxStates states: a move of a set S on class k
    // is follow(S) & mask(k), follow(S) the union of follow(q) over q in S
    // (a position automaton enters state p only on p's symbols).
    uint32_t nfa_words = 0;               // 64-bit words of a set (1, 2 or 4); 0 = too many states
    std::vector<uint64_t> nfa_follow;     // [n][nfa_words]
    std::vector<uint64_t> nfa_mask;       // [K][nfa_words]
};

constexpr uint32_t kNfaMaxStates = 256;

// Throws BuildError (RI_ERR_PARSE / RI_ERR_LIMIT).
void build_automata(const std::string &re, uint32_t max_states, Automata &out);

}  // namespace ri
