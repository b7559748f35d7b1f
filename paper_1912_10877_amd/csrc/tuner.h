// Timing of candidate schedules: the fusion width of forward sweeps and the tile sizes of the
// tile passes are picked by running each candidate on the device and keeping the fastest.
#pragma once

#include "fused.h"

namespace yao {

// A program copied to a private device buffer (trial runs do not touch the shared workspace).
struct TrialProgram {
    char* d = nullptr;
    DevProgram dp{};
    TrialProgram() = default;
    TrialProgram(const TrialProgram&) = delete;
    TrialProgram& operator=(const TrialProgram&) = delete;
    ~TrialProgram();
    int load(const Program& p);  // ordered on the current stream; synchronises it
};

// Median GPU time in ms of `reps` runs of fn (after one untimed run), measured with events
// on the current stream. fn returns a status.
int time_runs(int reps, int (*fn)(void*), void* ctx, double* ms);
template <typename F> int time_ms(int reps, F&& f, double* ms)
{
    return time_runs(reps, [](void* p) { return (*(F*)p)(); }, (void*)&f, ms);
}

// The circuit a forward sweep runs at fusion width w (0: c itself; 1: runs of one-qubit gates
// merged; 2..5: dense blocks of up to w qubits), its matrices refreshed for params. *fparams
// receives the parameters that circuit takes (params, or null for a fused circuit).
const yao_circuit* forward_circuit(const yao_circuit* c, const double* params, int width, const double** fparams);

// GPU time of the fused forward sweep of c at fusion width `width` and tile qubits tq on data
// (overwritten).
int time_forward(const yao_circuit* c, const double* params, void* data, int dtype, int n, int B, int width, int tq,
                 double* ms);

// Fusion width for the forward sweep of c on states of this shape: options().fuse_width, or,
// with options().autotune, the fastest candidate, timed on data the first time (data is
// restored afterwards).
int pick_forward_width(const yao_circuit* c, const double* params, void* data, int dtype, int n, int B, int* width);
void drop_tuning(const yao_circuit* c);

}  // namespace yao
